// Kernels of one time step.
//
// State between steps: buffer `cur` holds the post-collision populations
// f*(t) in structure-of-arrays layout, nine planes of ny rows of `pitch`
// elements.  A step is two launches:
//
//   k_boundary(cur): one lane per cut link evaluates the wall rule
//     (Eqs. 7-14) from f*(t) and the node's saved moments; the first lane
//     of each boundary node then forms the node's sums for scheme B or Bao
//     and the leak of Eq. (15) for scheme A.  Each incoming population is
//     written into the solid neighbour's slot of the opposite direction
//     (the "ghost" slot: the only slot a pull from the fluid node reads
//     there).  Scheme A adds the leak to the node's own rest population.
//     Each block also sums the momentum its links hand to the wall; with
//     open x boundaries, further blocks set the inlet and outlet columns.
//
//   k_main(cur -> nxt): pull-streaming (Eq. 3) of all nine populations,
//     density, pseudopotential, the force of Eq. (16), the velocity of
//     Eq. (5) and collision (Eq. 2), fused.  A workgroup owns a strip of
//     tile_w columns and marches through tile_h rows, keeping psi of three
//     consecutive rows in a four-slot LDS ring; the loads of the next two
//     rows are in flight while a row is computed, and the first wavefront
//     also pulls the strip's two halo columns.  Solid nodes are not
//     stored.  Boundary nodes (and the x_f nodes that MLS reads) save their
//     moments, and under Zhao-Yong their pre-collision populations, for the
//     next k_boundary.  Each workgroup writes one FP64 partial of the total
//     mass; the next launch reduces the partials in a fixed order.
#pragma once

#include "lattice.hpp"

namespace lbm {

constexpr int kMaxTileW = 256;

enum : uint8_t { FL_SOLID = 1, FL_SAVE_MOM = 2, FL_SAVE_F = 4 };

// Workgroups are handed to the 8 XCDs round robin.  Give XCD k a
// contiguous run of tiles, numbered segment-major (all strips of a band of
// rows), so that the workgroups that run together on one XCD cover a
// compact block of the lattice and find each other's halo rows and columns
// in that XCD's L2.
__host__ __device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int xcd = b & 7, idx = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename S>
struct MainArgs {
    const S* __restrict__ src;
    S* __restrict__ dst;
    const uint8_t* __restrict__ flags;  // per node (pitch layout)
    const int* __restrict__ side_idx;   // per node, flagged only
    const float* __restrict__ psiw;     // FP16 storage: psi_w of solid nodes
    double* __restrict__ side_mom;      // [slot][3]: rho, ux, uy
    double* __restrict__ side_f;        // [slot][9]: pre-collision f
    double* __restrict__ partial;       // per workgroup
    double* __restrict__ mom_out;       // moments mode: rho, ux, uy planes
    int nx, ny, pitch;
    long long plane;                    // elements per population plane
    int tile_h, nsegs, nstrips;
    unsigned side_mom_bytes, side_f_bytes;
};

// Buffer resources: a 32-bit byte range on an SGPR base, so that a load
// needs no per-lane address arithmetic (row offset in an SGPR, column
// offset in a VGPR) and an access outside the range reads 0.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kRsrcWord3);
}
// A lane offset at or beyond every buffer's range: the access is dropped.
// Buffers stay below kOOB bytes.
constexpr unsigned kOOB = 0xFFFFFF00u;

template <typename T>
__device__ __forceinline__ T bload(rsrc_t r, unsigned v, unsigned s);
template <>
__device__ __forceinline__ int bload<int>(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
}
template <>
__device__ __forceinline__ float bload<float>(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
template <>
__device__ __forceinline__ double bload<double>(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
template <>
__device__ __forceinline__ _Float16 bload<_Float16>(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
}
template <>
__device__ __forceinline__ uint8_t bload<uint8_t>(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, v, s, 0);
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, 0);
}
__device__ __forceinline__ void bstore(_Float16 x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, 0);
}
__device__ __forceinline__ void bstore(double x, rsrc_t r, unsigned v, unsigned s) {
    typedef __attribute__((ext_vector_type(2))) unsigned u2;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, v, s, 0);
}

template <typename R>
__device__ __forceinline__ R dens(const R f[9]) {
    return ((f[0] + (f[1] + f[3])) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
}

// One row of a strip in flight, in the storage type: the pulled populations
// of the thread's column with its flags and (solid nodes) the wall psi.
template <typename S, typename R, int NR>
struct RowLoad {
    S f[9];
    uint8_t fl;
    int si;        // side slot (boundary nodes)
    float dr[NR];  // DEV 2: density two rows ahead, own column and edge column
    float rr[9];   // DEV 2: densities of the nine source nodes
    float pw;      // FP16 storage: psi_w of a solid node in FP32
};

// Density, force and velocity of one node from its pulled populations fc
// (stored form: f, or with DEV 1 the deviations from w rho_ref) and the
// psi of the node and its neighbours ps[a] = psi(x + e_a):
//   rho = sum f (Eq. 5); F = -G psi(x) sum_a w_a psi(x + e_a) e_a (Eq. 16),
//   opposite neighbours paired, plus rho g; u = (sum f e + F/2) / rho (Eq. 5).
template <typename R, int EOS, int DEV>
__device__ __forceinline__ void node_moments(const R fc[9], const R ps[9], const Phys<R>& ph,
                                             R& rho, R& drho, R& ux, R& uy, R& Fx, R& Fy) {
    drho = dens<R>(fc);
    rho = DEV == 1 ? ph.rref + drho : drho;
    const R irho = rcp(rho);
    Fx = R(0);
    Fy = R(0);
    if constexpr (EOS != EOS_NONE) {
        const R w1 = R(wf(1)), w5 = R(wf(5));
        const R sx = fma(w1, ps[1] - ps[3], w5 * ((ps[5] - ps[7]) + (ps[8] - ps[6])));
        const R sy = fma(w1, ps[2] - ps[4], w5 * ((ps[5] - ps[7]) + (ps[6] - ps[8])));
        const R g = -ph.G * ps[0];
        Fx = g * sx;
        Fy = g * sy;
    }
    Fx = fma(rho, ph.gx, Fx);
    Fy = fma(rho, ph.gy, Fy);
    const R mx = (fc[1] - fc[3]) + ((fc[5] - fc[7]) + (fc[8] - fc[6]));
    const R my = (fc[2] - fc[4]) + ((fc[5] - fc[7]) + (fc[6] - fc[8]));
    ux = fma(R(0.5), Fx, mx) * irho;
    uy = fma(R(0.5), Fy, my) * irho;
}

// Columns a strip updates: a workgroup of tile_w lanes also pulls the
// column on either side of its strip, for psi only.
__host__ __device__ constexpr int strip_cols(int tile_w) { return tile_w - 2; }

// One tile of the main pass: strip `strip` (at most strip_cols(blockDim.x)
// columns, plus one psi-only column on each side), rows of segment `seg`.
// Writes the tile's mass partial to partial[tile].
// MOMENTS: write rho, u at every node instead of colliding and storing.
// DEV: 0 populations stored as they are; 1 as deviations g = f - w rho_ref
// from one reference density; 2 as deviations g = f - w r(x) from the
// density r(x) of the node x whose slot holds g, kept in an FP32 plane
// after the nine population planes of each buffer.
// SAVEF: boundary nodes also save their pre-collision populations.
//
// Every lane issues every load and store of every row, so the number of
// memory operations in flight is the same on all paths and the waits
// before a use are exact: the rows in flight keep streaming while a row is
// computed.  A lane with nothing to move passes an offset beyond the
// buffer's range, which the hardware drops (no memory access; a load
// returns 0).  Solid nodes keep psi of their wall density in their own
// rest slot (plane 0), which nothing else reads or writes; with FP16
// storage it is read in FP32 from a per-node array instead.
template <typename S, typename R, int EOS, bool MOMENTS, int DEV, bool SAVEF, int RING = 3>
__device__ __forceinline__ void main_tile(const MainArgs<S>& a, const Phys<R>& ph,
                                          int tile) {
    // RING rows of loads: RING - 1 rows are in flight while a row is
    // computed (the FP16 per-node form's density ring assumes three)
    static_assert(RING >= 2 && RING <= 4 && (DEV != 2 || RING == 3), "unsupported ring");
    __shared__ R ring[4][kMaxTileW];
    __shared__ double wsum[kMaxTileW / 64];
    constexpr unsigned ES = sizeof(S);
    // DEV 2: the density plane's rows -2 .. H + 1 of the strip, with one
    // column more on either side, pass through an LDS ring of eight rows:
    // row j is loaded with row j - 2's populations, written at row j - 3's
    // step and read by the decodes of rows j - 1 .. j + 1
    constexpr int NR = DEV == 2 ? 2 : 1;
    __shared__ float dring[DEV == 2 ? 8 : 1][kMaxTileW + 2];
    const unsigned pitch = (unsigned)a.pitch;
    // one resource per buffer; plane and row offsets go in the scalar
    // offset (the whole buffer is below 4 GiB)
    const unsigned pb = (unsigned)(a.plane * ES);
    const unsigned bbytes = 9u * pb + (DEV == 2 ? (unsigned)a.plane * 4u : 0u);
    const rsrc_t rs = make_rsrc(a.src, bbytes);
    const rsrc_t rd = make_rsrc(a.dst, bbytes);
    const rsrc_t rfl = make_rsrc(a.flags, pitch * (unsigned)a.ny);
    const rsrc_t rsi = make_rsrc(a.side_idx, pitch * (unsigned)a.ny * 4u);
    const rsrc_t rsm = make_rsrc(a.side_mom, a.side_mom_bytes);
    const rsrc_t rsf = make_rsrc(a.side_f, a.side_f_bytes);
    const rsrc_t rpw = make_rsrc(a.psiw, ES == 2 ? pitch * (unsigned)a.ny * 4u : 0u);
    // DEV 2: the FP32 density plane follows the nine population planes
    const unsigned rbase = 9u * pb;

    const int tid = threadIdx.x;
    const int W = blockDim.x;
    const int seg = tile / a.nstrips, strip = tile - seg * a.nstrips;
    // the nstrips = ceil(nx / strip_cols) strips share the columns evenly
    const int x0 = (int)(((unsigned long long)strip * (unsigned)a.nx) / (unsigned)a.nstrips);
    const int ncols =
        (int)(((unsigned long long)(strip + 1) * (unsigned)a.nx) / (unsigned)a.nstrips) - x0;
    // lane t pulls column x0 - 1 + t; lanes 1..ncols update theirs, lanes 0
    // and ncols + 1 only supply psi, the rest are idle
    const bool act = tid <= ncols + 1;
    const bool upd = tid >= 1 && tid <= ncols;
    int xi = x0 - 1 + (act ? tid : 1);
    xi = xi < 0 ? xi + a.nx : (xi >= a.nx ? xi - a.nx : xi);
    const unsigned x = (unsigned)xi;
    const unsigned xm = x == 0 ? a.nx - 1 : x - 1;
    const unsigned xp = x == (unsigned)a.nx - 1 ? 0 : x + 1;
    // rows: even segments march up, odd ones down, so that neighbouring
    // segments reach their shared boundary rows at the same time
    const int y0 = seg * a.tile_h;
    const int H = min(a.tile_h, a.ny - y0);
    const int dir = (seg & 1) ? -1 : 1;
    const int ystart = dir > 0 ? y0 : y0 + H - 1;
    auto row_of = [&](int k) {
        int y = ystart + dir * k;
        y = y < 0 ? y + a.ny : y;
        y = y >= a.ny ? y - a.ny : y;
        return y;
    };

    // flags of the next row to issue are loaded one issue ahead
    uint8_t nfl;
    auto load_flags = [&](int k) {
        nfl = bload<uint8_t>(rfl, x, (unsigned)row_of(k) * pitch);
    };
    // DEV 2: density row j of the ring (-2 <= j <= H + 1), own column, and
    // for lanes 0 and ncols + 1 the column beyond
    auto load_dens = [&](int j, RowLoad<S, R, NR>& L) {
        const bool in = j >= -2 && j <= H + 1;
        const unsigned q = rbase + (unsigned)(in ? row_of(j) : 0) * pitch * 4u;
        L.dr[0] = bload<float>(rs, (in && act) ? x * 4u : kOOB, q);
        const unsigned xe = tid == 0 ? xm : xp;
        L.dr[1 % NR] = bload<float>(rs, (in && (tid == 0 || tid == ncols + 1)) ? xe * 4u : kOOB, q);
    };
    auto put_dens = [&](int j, const RowLoad<S, R, NR>& L) {
        // lane t's column sits at t + 1; idle lanes write nothing
        float* const d = dring[j & 7];
        if (act) d[tid + 1] = L.dr[0];
        if (tid == 0) d[0] = L.dr[1 % NR];
        if (tid == ncols + 1) d[ncols + 3] = L.dr[1 % NR];
    };
    // DEV 2: densities of the nine nodes row k pulls from (0 where the node
    // itself is not fluid); x - e_q lies in column tid + 1 - e_qx of the
    // ring and in row k - e_qy * dir
    auto src_dens = [&](int k, uint8_t fl, float rr[9]) {
        const bool fluid = !(fl & FL_SOLID);
        const float* const dm = dring[(k - dir) & 7];
        const float* const d0 = dring[k & 7];
        const float* const dp = dring[(k + dir) & 7];
        rr[0] = d0[tid + 1];
        rr[1] = d0[tid];
        rr[2] = dm[tid + 1];
        rr[3] = d0[tid + 2];
        rr[4] = dp[tid + 1];
        rr[5] = dm[tid];
        rr[6] = dm[tid + 2];
        rr[7] = dp[tid + 2];
        rr[8] = dp[tid];
#pragma unroll
        for (int q = 0; q < 9; ++q) rr[q] = fluid ? rr[q] : 0.0f;
    };
    // rows -1 .. H are pulled (the outer two for psi only); later ones only
    // keep the pipeline uniform and move nothing
    auto issue = [&](int k, RowLoad<S, R, NR>& L) {
        const int y = row_of(k);
        const bool rv = k <= H;
        const uint8_t fl = (act && rv) ? nfl : uint8_t(FL_SOLID);
        L.fl = fl;
        load_flags(k + 1);
        const bool own = act && rv, fluid = !(fl & FL_SOLID);
        const unsigned r0 = (unsigned)y * pitch * ES;
        const unsigned rm = (unsigned)(y == 0 ? a.ny - 1 : y - 1) * pitch * ES;
        const unsigned rp = (unsigned)(y == a.ny - 1 ? 0 : y + 1) * pitch * ES;
        const unsigned vc = fluid ? x * ES : kOOB, vm = fluid ? xm * ES : kOOB,
                       vp = fluid ? xp * ES : kOOB;
        // plane 0 of the node itself: the rest population, or psi_w if solid
        L.f[0] = bload<S>(rs, own ? x * ES : kOOB, r0);
        L.f[1] = bload<S>(rs, vm, 1 * pb + r0);
        L.f[2] = bload<S>(rs, vc, 2 * pb + rm);
        L.f[3] = bload<S>(rs, vp, 3 * pb + r0);
        L.f[4] = bload<S>(rs, vc, 4 * pb + rp);
        L.f[5] = bload<S>(rs, vm, 5 * pb + rm);
        L.f[6] = bload<S>(rs, vp, 6 * pb + rm);
        L.f[7] = bload<S>(rs, vp, 7 * pb + rp);
        L.f[8] = bload<S>(rs, vm, 8 * pb + rp);
        if constexpr (DEV == 2) load_dens(k + 2, L);
        if constexpr (ES == 2)
            L.pw = bload<float>(rpw, (own && !fluid) ? x * 4u : kOOB, (unsigned)y * pitch * 4u);
        if constexpr (!MOMENTS) {
            // side slot of a boundary node (or of an x_f node of MLS)
            // (a wavefront with no such node in the row issues nothing)
            const bool side = fluid && (fl & (FL_SAVE_MOM | FL_SAVE_F));
            L.si = 0;
            if (__builtin_amdgcn_ballot_w64(side))
                L.si = bload<int>(rsi, side ? x * 4u : kOOB, (unsigned)y * pitch * 4u);
        }
    };
    // stored form -> populations (DEV 2, with the source densities rr) or
    // the stored form itself.  DEV 2 fuses the multiply-add explicitly: the
    // row loop's unrolled copies must round alike whatever the compiler
    // would contract in each
    auto decode = [&](const RowLoad<S, R, NR>& L, const float rr[9], R f[9]) {
#pragma unroll
        for (int q = 0; q < 9; ++q)
            f[q] = DEV == 2 ? fma(R(wt(q)), R(rr[q]), R(L.f[q])) : R(L.f[q]);
    };
    // psi of row k into ring slot (k + 1) & 3 (DEV 2: with the source
    // densities of the row, kept for its collision)
    auto publish = [&](RowLoad<S, R, NR>& L, int k) {
        const int slot = (k + 1) & 3;
        if constexpr (DEV == 2) src_dens(k, L.fl, L.rr);
        R f[9];
        decode(L, L.rr, f);
        const R rho = DEV == 1 ? ph.rref + dens<R>(f) : dens<R>(f);
        const R pw = ES == 2 ? R(L.pw) : R(L.f[0]);
        ring[slot][tid] = (L.fl & FL_SOLID) ? pw : psi_of<EOS, R>(rho, ph);
    };

    double msum = 0.0;
    // row k: collide with psi of rows k-1, k, k+1; then prefetch row k+3
    auto step = [&](int k, RowLoad<S, R, NR>& Lc, RowLoad<S, R, NR>& Ln) {
        const int y = row_of(k);
        const int sm = k & 3, s0 = (k + 1) & 3, sp = (k + 2) & 3;
        const int sym = dir > 0 ? sm : sp, syp = dir > 0 ? sp : sm;
        if constexpr (DEV == 2) put_dens(k + 3, Ln);
        publish(Ln, k + 1);
        __syncthreads();
        const bool live = upd && k < H && !(Lc.fl & FL_SOLID);
        const float* const rr = Lc.rr;
        R fc[9];  // f, or (DEV 1) the deviations g
        decode(Lc, rr, fc);
        const int c = tid;
        // psi of the node and of its eight neighbours, by direction
        const int cl = c > 0 ? c - 1 : 0, cr = c < W - 1 ? c + 1 : W - 1;
        const R ps[9] = {ring[s0][c],    ring[s0][cr],   ring[syp][c],
                         ring[s0][cl],   ring[sym][c],   ring[syp][cr],
                         ring[syp][cl],  ring[sym][cl],  ring[sym][cr]};
        R rho, drho, ux, uy, Fx, Fy;
        node_moments<R, EOS, DEV>(fc, ps, ph, rho, drho, ux, uy, Fx, Fy);
        if constexpr (MOMENTS) {
            if (upd && k < H) {
                const bool fl = live;
                const long long o = (long long)y * a.nx + x;
                const long long n2 = (long long)a.nx * a.ny;
                a.mom_out[o] = fl ? (DEV == 1 ? double(ph.rref) + double(drho) : double(rho)) : 0.0;
                a.mom_out[n2 + o] = fl ? double(ux) : 0.0;
                a.mom_out[2 * n2 + o] = fl ? double(uy) : 0.0;
            }
        } else {
            // FP64 density (the deviation forms add the reference here)
            double rho_d = DEV == 1 ? double(ph.rref) + double(drho) : double(rho);
            if constexpr (DEV == 2) {
                rho_d = 0.0;
#pragma unroll
                for (int q = 0; q < 9; ++q) rho_d += fma(wt(q), double(rr[q]), double(Lc.f[q]));
            }
            msum += live ? rho_d : 0.0;
            // moments of boundary nodes (and pre-collision populations)
            // (stores only from a wavefront with such a node in the row:
            // the branch is uniform, and the waits for the rows in flight
            // stay exact on the path without them)
            const bool sm = live && (Lc.fl & FL_SAVE_MOM);
            if (__builtin_amdgcn_ballot_w64(sm)) {
                const unsigned so = sm ? (unsigned)Lc.si * 24u : kOOB;
                bstore(rho_d, rsm, so, 0u);
                bstore(double(ux), rsm, so + 8u, 0u);
                bstore(double(uy), rsm, so + 16u, 0u);
            }
            if constexpr (SAVEF) {
                const bool sf = live && (Lc.fl & FL_SAVE_F);
                if (__builtin_amdgcn_ballot_w64(sf)) {
                    const unsigned fo = sf ? (unsigned)Lc.si * 72u : kOOB;
#pragma unroll
                    for (int q = 0; q < 9; ++q)
                        bstore(DEV == 1 ? double(fc[q]) + wt(q) * double(ph.rref) : double(fc[q]),
                               rsf, fo + 8u * q, 0u);
                }
            }
            R dh[9];
            collide<R>(fc, rho, drho, ux, uy, Fx, Fy, ph, dh);
            const unsigned r0 = (unsigned)y * pitch * ES;
            const unsigned vo = live ? x * ES : kOOB;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                // DEV 2: re-encoded against this node's density,
                // g* = g + w (r(x - e) - rho) + dh, without forming f
                const R v = DEV == 2 ? fma(R(wt(q)), R(rr[q]) - rho, R(Lc.f[q])) + dh[q]
                                     : fc[q] + dh[q];
                bstore(S(v), rd, vo, q * pb + r0);
            }
            if constexpr (DEV == 2)
                bstore(float(rho), rd, live ? x * 4u : kOOB, rbase + (unsigned)y * pitch * 4u);
        }
        issue(k + RING, Lc);  // Lc is free again
    };

    RowLoad<S, R, NR> L[RING];
    // DEV 2: density rows -2 .. 0 here, 1 and 2 with the first two issues
    RowLoad<S, R, NR> D0, D1, D2;
    if constexpr (DEV == 2) {
        load_dens(-2, D0);
        load_dens(-1, D1);
        load_dens(0, D2);
    }
    load_flags(-1);
    issue(-1, L[RING - 1]);
#pragma unroll
    for (int i = 0; i + 1 < RING; ++i) issue(i, L[i]);
    if constexpr (DEV == 2) {
        put_dens(-2, D0);
        put_dens(-1, D1);
        put_dens(0, D2);
        put_dens(1, L[2]);
        put_dens(2, L[0]);
        __syncthreads();
    }
    publish(L[RING - 1], -1);
    issue(RING - 1, L[RING - 1]);
    publish(L[0], 0);
    // a whole number of ring rotations; rows k >= H store nothing
    const int HR = (H + RING - 1) / RING * RING;
    for (int k = 0; k < HR; k += RING) {
#pragma unroll
        for (int i = 0; i < RING; ++i) step(k + i, L[i], L[(i + 1) % RING]);
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
            a.partial[tile] = t;
        }
    }
}

template <typename S, typename R, int EOS, bool MOMENTS, int DEV, bool SAVEF>
__global__ __launch_bounds__(256) void k_main(MainArgs<S> a, Phys<R> ph) {
    main_tile<S, R, EOS, MOMENTS, DEV, SAVEF>(a, ph, xcd_tile(blockIdx.x, gridDim.x));
}

// Sum the main kernel's partials in a fixed order; the total lands in
// thread 0.
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int np) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    // each thread adds partials tid, tid + 256, ... in that order; eight
    // loads are issued before their additions
    double v = 0.0;
    int i = tid;
    for (; i + 7 * 256 < np; i += 8 * 256) {
        double q[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = partial[i + j * 256];
#pragma unroll
        for (int j = 0; j < 8; ++j) v += q[j];
    }
    for (; i < np; i += 256) v += partial[i];
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    return red[0];
}

// The total into hist[slot], and the first non-finite one into unstable.
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partial,
                                                int np, double* __restrict__ hist,
                                                long long slot, long long t,
                                                long long* __restrict__ unstable) {
    const double m = sum_partials(partial, np);
    if (threadIdx.x == 0) {
        hist[slot] = m;
        if (!isfinite(m) && *unstable < 0) *unstable = t;
    }
}

// As reduce_partials, with the step taken from a device clock that holds
// the step of the last recorded mass and advances by one: the launches of
// a step then need no argument that changes from step to step, so a
// captured graph of steps can be replayed.
__device__ __forceinline__ void reduce_on_clock(const double* __restrict__ partial, int np,
                                                double* __restrict__ hist, long long cap,
                                                long long* __restrict__ clock,
                                                long long* __restrict__ unstable) {
    const double m = sum_partials(partial, np);
    if (threadIdx.x == 0) {
        const long long t = *clock + 1;
        hist[t % cap] = m;
        if (!isfinite(m) && *unstable < 0) *unstable = t;
        *clock = t;
    }
}

// The masses of the last pass: one step (partial2 null) or two steps per
// pass (partial, then partial2), each recorded at the next step of the clock.
__device__ __forceinline__ void reduce_pass(const double* __restrict__ partial,
                                            const double* __restrict__ partial2, int np,
                                            double* __restrict__ hist, long long cap,
                                            long long* __restrict__ clock,
                                            long long* __restrict__ unstable) {
    reduce_on_clock(partial, np, hist, cap, clock, unstable);
    if (partial2) {
        __syncthreads();  // every thread has read the first total
        reduce_on_clock(partial2, np, hist, cap, clock, unstable);
    }
}

template <int Unused = 0>
__global__ __launch_bounds__(256) void k_reduce(const double* partial, const double* partial2,
                                                int np, double* hist, long long cap,
                                                long long* clock, long long* unstable) {
    reduce_pass(partial, partial2, np, hist, cap, clock, unstable);
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

// One lane per cut link.  Links are grouped by boundary node (directions
// ascending) and the groups are padded so that none straddles a
// workgroup; per-node sums are taken by the group's first lane from LDS in
// link order.
struct BndArgs {
    int nslot;                       // link slots, padding included
    const int* __restrict__ lnode;   // x_b (pitch layout)
    const int* __restrict__ lmeta;   // dir | kind << 4 | len << 8 | pos << 12
                                     // | (DEV 2: sets the ghost's density) << 16
    const int* __restrict__ lghost;  // solid neighbour x_s
    const int* __restrict__ lxf;     // x_f (or -1)
    const int* __restrict__ lxff;    // x_ff (or -1)
    const int* __restrict__ lslotb;  // side slot of x_b
    const int* __restrict__ lslotf;  // side slot of x_f (or -1)
    const double* __restrict__ lc;   // [slot][8]: c1 c2 c3 chi cb uwq_x uwq_y pad
    const double* __restrict__ luw;  // [slot][2]: wall velocity
    const double* __restrict__ side_mom;
    const double* __restrict__ side_f;
    long long plane;
    double rref;                     // deviation storage reference (else 0)
    const int* __restrict__ lref;    // DEV 2: side slot whose density encodes
                                     // the ghost (one boundary node per ghost)
    int fix;                         // 0 none, 1 A, 2 B, 3 Bao
    // reduction of the previous main launch's mass partials (last block):
    // one array per step of that launch (partial2 null for a single step)
    const double* __restrict__ partial;
    const double* __restrict__ partial2;
    int np;
    double* __restrict__ hist;
    long long cap;                   // history ring entries
    long long* __restrict__ clock;   // step of the last recorded mass
    long long* __restrict__ unstable;
    int do_reduce;
    // force on the walls (Sec. 4.2, momentum exchange): two FP64 partials
    // per link block (null: not formed)
    double* __restrict__ force;
    // open x boundaries (Sec. 4.2): blocks nlink_blocks .. of the grid take
    // one row each lane
    int nlink_blocks;
    int open_x;
    int nx, ny, pitch;
    double inlet_u;
    // scheme A: count of boundary nodes whose rest population came out
    // negative (null: not counted)
    unsigned long long* __restrict__ negrest;
    // scheme B / Bao: count of boundary nodes whose sums in Eq. (22) or
    // (23) cancel, which keep rho_b (null: not counted)
    unsigned long long* __restrict__ degen;
};

constexpr int LK_PAD = 15;

// Inputs of a wall rule besides f*_a(x_b) and the node's own moments,
// fetched only by the kinds that use them.
enum : int { LV_OD_B, LV_D_F, LV_D_FF, LV_OD_F, LV_PRE, LV_UFX, LV_UFY };

// The incoming population f_abar(x_b, t + 1) of one cut link (x_b, a) from
// its kind and coefficients c (table layout of BndArgs::lc), the wall
// velocity uw, f*_a(x_b, t) = fab and the node's moments rho_b, u_b;
// fetch(LV_*) supplies the other populations and u_f.  Also returns chi
// (ch), the bracket of Eq. (8) (bk) and the moving-wall term (wl), which
// schemes A and B need.  The one evaluation of every rule: both the
// boundary pass and the two-steps-per-pass kernel call it, so both round
// every rule alike.
template <typename F>
__device__ __forceinline__ double link_value(int kind, int d, const double* c, double uwx,
                                             double uwy, double fab, double rho_b, double ubx,
                                             double uby, double& ch, double& bk, double& wl,
                                             F&& fetch) {
    const double ex = double(cx(d)), ey = double(cy(d));
    // momentum of a moving wall, Ladd / Mei et al.: 2 w_a rho_b e.u_w / c_s^2
    wl = 2.0 * wt(d) * rho_b * 3.0 * (ex * uwx + ey * uwy);
    ch = 0.0;
    bk = 0.0;
    if (kind == LK_HALFWAY) return fab - wl;
    if (kind <= LK_CHI_EXT) {
        double usx, usy;
        if (kind == LK_CHI_UB) {
            usx = ubx;
            usy = uby;
        } else if (kind == LK_CHI_UF) {
            usx = fetch(LV_UFX);
            usy = fetch(LV_UFY);
        } else {
            usx = c[4] * ubx + c[5];
            usy = c[4] * uby + c[6];
        }
        ch = c[3];
        // Eq. (8): w_a [1 + 3 e.u_s + 4.5 (e.u_b)^2 - 1.5 u_b^2]
        const double eus = edot<double>(d, usx, usy);
        const double eub = edot<double>(d, ubx, uby);
        const double ub2 = ubx * ubx + uby * uby;
        bk = wt(d) * (1.0 + 3.0 * eus + 4.5 * (eub * eub) - 1.5 * ub2);
        return (1.0 - ch) * fab + ch * (rho_b * bk) - wl;  // Eq. (7)
    }
    if (kind == LK_LIN_F) return c[0] * fab + c[1] * fetch(LV_D_F);
    if (kind == LK_LIN_B) return c[0] * fab + c[1] * fetch(LV_OD_B);
    if (kind == LK_QUAD_F) return c[0] * fab + c[1] * fetch(LV_D_F) - c[2] * fetch(LV_D_FF);
    if (kind == LK_QUAD_B) return c[0] * fab + c[1] * fetch(LV_OD_B) - c[2] * fetch(LV_OD_F);
    return c[0] * fetch(LV_OD_B) + c[1] * fetch(LV_PRE);  // LK_ZY, Eq. (14)
}

// Block `blk` of 256 link slots.
template <typename S, int DEV>
__device__ __forceinline__ void boundary_block(S* __restrict__ A, const BndArgs& b,
                                               int blk) {
    __shared__ double s_fab[256], s_inc[256], s_chi[256], s_br[256], s_wall[256];
    __shared__ double s_rhos[256];
    const int tid = threadIdx.x;
    const int i = blk * 256 + tid;
    const int meta = i < b.nslot ? b.lmeta[i] : (LK_PAD << 4);
    const int d = meta & 15, kind = (meta >> 4) & 15;
    const int len = (meta >> 8) & 15, pos = (meta >> 12) & 15;
    const bool active = kind != LK_PAD;
    const long long P = b.plane;
    // stored form -> population
    // DEV 2: densities of the nodes, after the nine population planes
    float* const rpl = reinterpret_cast<float*>(A + 9 * P);
    auto ld = [&](int q, int n) {
        if constexpr (DEV == 2) return double(A[q * P + n]) + wt(q) * double(rpl[n]);
        return DEV == 1 ? double(A[q * P + n]) + wt(q) * b.rref : double(A[q * P + n]);
    };
    // the link's record, loaded beside its metadata (a padding slot of the
    // table stands in for the lanes past its end): one round trip fewer
    // before the populations
    const int ic = i < b.nslot ? i : 0;
    const int node_r = b.lnode[ic], slotb = b.lslotb[ic], slotf = b.lslotf[ic];
    const int xf = b.lxf[ic], xff = b.lxff[ic];
    // the ghost slot too (and, per-node references, the node whose density
    // encodes it), so that the final store waits for no load of its own
    const int ghost = b.lghost[ic];
    const int gref = DEV == 2 ? b.lref[ic] : 0;
    double c[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) c[k] = b.lc[8 * ic + k];
    const double uwx = b.luw[2 * ic], uwy = b.luw[2 * ic + 1];
    int node = 0;
    double fab = 0.0, r = 0.0, ch = 0.0, bk = 0.0, wl = 0.0;
    if (active) {
        node = node_r;
        const int od = opp(d);
        const double* mom = b.side_mom + 3 * slotb;
        fab = ld(d, node);
        r = link_value(kind, d, c, uwx, uwy, fab, mom[0], mom[1], mom[2], ch, bk, wl,
                       [&](int what) -> double {
                           switch (what) {
                           case LV_OD_B: return ld(od, node);
                           case LV_D_F: return ld(d, xf);
                           case LV_D_FF: return ld(d, xff);
                           case LV_OD_F: return ld(od, xf);
                           case LV_PRE: return b.side_f[9 * slotb + d];
                           case LV_UFX: return b.side_mom[3 * slotf + 1];
                           default: return b.side_mom[3 * slotf + 2];
                           }
                       });
    }
    s_fab[tid] = fab;
    s_inc[tid] = r;
    s_chi[tid] = ch;
    s_br[tid] = bk;
    s_wall[tid] = wl;
    __syncthreads();
    const bool head = active && pos == 0;
    const int h = tid - pos;
    if (b.fix == 2 || b.fix == 3) {
        // scheme B, Eq. 22 (chi inside the sums) or Bao et al., Eq. 23
        if (head) {
            double num = 0.0, den = 0.0, mag = 0.0;
            for (int m = 0; m < len; ++m) {
                if (b.fix == 2) {
                    num += s_chi[tid + m] * s_fab[tid + m];
                    den += s_chi[tid + m] * s_br[tid + m];
                    mag += fabs(s_chi[tid + m] * s_br[tid + m]);
                } else {
                    num += s_fab[tid + m];
                    den += s_br[tid + m];
                    mag += fabs(s_br[tid + m]);
                }
            }
            const bool ok = den != 0.0 && fabs(den) > 1e-12 * mag;
            s_rhos[tid] = ok ? num / den : NAN;
            // (a node whose every chi is 0 has no leak and is not counted)
            if (!ok && mag > 0.0 && b.degen) atomicAdd(b.degen, 1ull);
        }
        __syncthreads();
        if (active) {
            const double rho_s = s_rhos[h];
            if (!isnan(rho_s)) {
                r = (1.0 - ch) * fab + ch * (rho_s * bk) - wl;
                s_inc[tid] = r;
            }
        }
        __syncthreads();
    }
    if (active) {
        const int g = ghost;
        double enc = DEV == 1 ? wt(d) * b.rref : 0.0;
        if constexpr (DEV == 2) {
            // every link into ghost g encodes against the same density: that
            // of one boundary node next to it, which one of them records
            const float rg = float(b.side_mom[3 * gref]);
            if ((meta >> 16) & 1) rpl[g] = rg;
            enc = wt(d) * double(rg);
        }
        A[opp(d) * P + g] = S(r - enc);
    }
    if (head && b.fix == 1) {
        // Eq. (15) without the wall momentum, added to the rest population
        // (Eq. 18)
        double out_sum = 0.0, in_sum = 0.0;
        for (int m = 0; m < len; ++m) {
            out_sum += s_fab[tid + m];
            in_sum += s_inc[tid + m] + s_wall[tid + m];
        }
        const double v = double(A[node]) + (out_sum - in_sum);
        A[node] = S(v);
        if (b.negrest) {
            // Eq. (18) can leave the rest population negative: counted,
            // not clamped
            double f0 = v;
            if constexpr (DEV == 2) f0 += wt(0) * double(rpl[node]);
            if constexpr (DEV == 1) f0 += wt(0) * b.rref;
            if (f0 < 0.0) atomicAdd(b.negrest, 1ull);
        }
    }
    if (b.force) {
        // momentum handed to the wall by this link, e_a (f*_a + f_abar(t+1)),
        // summed in a fixed order: down each wavefront, then the four
        // wavefront sums
        __shared__ double s_fx[4], s_fy[4];
        const double m = fab + r;
        double vx = active ? double(cx(d)) * m : 0.0;
        double vy = active ? double(cy(d)) * m : 0.0;
        for (int off = 32; off > 0; off >>= 1) {
            vx += __shfl_down(vx, off, 64);
            vy += __shfl_down(vy, off, 64);
        }
        if ((tid & 63) == 0) {
            s_fx[tid >> 6] = vx;
            s_fy[tid >> 6] = vy;
        }
        __syncthreads();
        if (tid == 0) {
            b.force[2 * blk] = (s_fx[0] + s_fx[1]) + (s_fx[2] + s_fx[3]);
            b.force[2 * blk + 1] = (s_fy[0] + s_fy[1]) + (s_fy[2] + s_fy[3]);
        }
    }
}

// Open x boundaries (Sec. 4.2), lane y of block `blk` takes row y.  The
// seam between columns nx-1 and 0 is cut: the populations a node there
// pulls across it are written into the slots it pulls them from.
//   inlet, x = 0: velocity (U, 0) by the scheme of Zou and He (1997); the
//     node's density follows from the six populations that arrive from the
//     interior, and f1, f5, f8 are set so that its moments give (U, 0).
//   outlet, x = nx - 1: fully developed flow, f3, f6, f7 equal to those of
//     the node at nx - 2.
// No cut link reads or writes these slots (the three outermost columns on
// each side are fluid), so the rows run beside the link blocks.
template <typename S, int DEV>
__device__ __forceinline__ void open_rows(S* __restrict__ A, const BndArgs& b, int blk) {
    const int y = blk * 256 + int(threadIdx.x);
    if (y >= b.ny) return;
    const long long P = b.plane;
    float* const rpl = reinterpret_cast<float*>(A + 9 * P);
    auto ref = [&](int q, long long n) {
        if constexpr (DEV == 2) return wt(q) * double(rpl[n]);
        return DEV == 1 ? wt(q) * b.rref : 0.0;
    };
    auto ld = [&](int q, long long n) { return double(A[q * P + n]) + ref(q, n); };
    auto st = [&](int q, long long n, double v) { A[q * P + n] = S(v - ref(q, n)); };
    const long long p = b.pitch, e = b.nx - 1;
    const long long r0 = y * p;
    const long long rm = (y == 0 ? b.ny - 1 : y - 1) * p;
    const long long rp = (y == b.ny - 1 ? 0 : y + 1) * p;
    // populations of (0, y) after streaming, each where the pull reads it
    const double f0 = ld(0, r0), f2 = ld(2, rm), f4 = ld(4, rp);
    const double f3 = ld(3, r0 + 1), f6 = ld(6, rm + 1), f7 = ld(7, rp + 1);
    const double U = b.inlet_u;
    const double rho = (f0 + f2 + f4 + 2.0 * (f3 + f6 + f7)) / (1.0 - U);
    const double h = 0.5 * (f2 - f4), s6 = 1.0 / 6.0 * rho * U;
    st(1, r0 + e, f3 + 2.0 / 3.0 * rho * U);
    st(5, rm + e, f7 - h + s6);
    st(8, rp + e, f6 + h + s6);
    // outlet: (nx-1, y) pulls f3, f6, f7 through (0, y), (0, y-1), (0, y+1);
    // lane y fills row y of the three planes
    st(3, r0, ld(3, r0 + e));
    st(6, r0, ld(6, r0 + e));
    st(7, r0, ld(7, r0 + e));
}

// The last block reduces the previous main pass's mass partials.
template <typename S, int DEV>
__global__ __launch_bounds__(256) void k_boundary(S* __restrict__ A, BndArgs b) {
    if (blockIdx.x == gridDim.x - 1) {
        if (b.do_reduce) reduce_pass(b.partial, b.partial2, b.np, b.hist, b.cap, b.clock, b.unstable);
        return;
    }
    if (int(blockIdx.x) >= b.nlink_blocks) {
        open_rows<S, DEV>(A, b, blockIdx.x - b.nlink_blocks);
        return;
    }
    boundary_block<S, DEV>(A, b, blockIdx.x);
}

// f(0) = f_eq(rho0, u0), stored where the first pull reads it:
// buffer[a][x - e_a] = f_a(0)(x)
template <typename S>
__global__ void k_init_scatter(S* __restrict__ B, const uint8_t* __restrict__ flags,
                               const double* __restrict__ rho0,
                               const double* __restrict__ ux0,
                               const double* __restrict__ uy0, int nx, int ny,
                               int pitch, long long plane, double rref,
                               const float* __restrict__ ref) {
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
        const double r0 = ref ? double(ref[ys * pitch + xs]) : rref;
        B[a * plane + ys * pitch + xs] = S(f - wt(a) * r0);
    }
}

// psi of the virtual wall density, kept in the rest slot (plane 0) of each
// solid node in both buffers
template <typename S, typename R, int EOS>
__global__ void k_psi_wall(S* __restrict__ b0, S* __restrict__ b1, float* __restrict__ pw32,
                           const double* __restrict__ rho_wall,
                           const uint8_t* __restrict__ flags, int nx, int ny,
                           int pitch, Phys<R> ph) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx || y >= ny) return;
    const int i = y * pitch + x;
    if (flags[i] & FL_SOLID) {
        const R p = psi_of<EOS, R>(R(rho_wall[y * nx + x]), ph);
        b0[i] = S(p);
        b1[i] = S(p);
        if (pw32) pw32[i] = float(p);
    }
}

// ---------------------------------------------------------------- batches
// Many independent instances advance together: per step one boundary
// launch over the link blocks of all instances, one main launch over the
// tiles of all instances and one launch that reduces each instance's mass
// partials.  Everything a launch needs about an instance lives in device
// memory (BInst, BState), so the launch arguments stay fixed while
// instances come and go, and a captured graph of steps can be replayed.

// What the kernels read about one instance.
struct BInst {
    void* f[2];  // state buffers; f[t & 1] holds f*(t)
    const uint8_t* flags;
    const int* side_idx;
    const float* psiw;
    double* side_mom;
    double* side_f;
    double* partial;  // one FP64 mass partial per tile
    int nx, ny, pitch, nsegs, nstrips, np;
    unsigned side_mom_bytes, side_f_bytes;
    long long plane;
    Phys<double> ph;
    // boundary tables (see BndArgs)
    int nslot, fix;
    const int *lnode, *lmeta, *lghost, *lxf, *lxff, *lslotb, *lslotf;
    const double *lc, *luw;
    double rref;
    const int* lref;
    double* hist;
    long long cap;
    long long* unstable;
};

// Time step of an instance and the steps it still has to run; an instance
// with remaining <= 0 is skipped by every launch.
struct BState {
    long long t;
    long long remaining;
};

// Ints between two queue heads of the persistent form: each head on a
// line of its own, so that the tickets of different queues (taken with
// device-scope atomics, which the XCDs' L2 caches do not hold) do not queue
// up on one line.
constexpr int kQueueStride = 64;

struct BatchArgs {
    const BInst* __restrict__ inst;
    BState* __restrict__ state;
    const int2* __restrict__ tiles;  // (instance, tile) in queue order
    int* __restrict__ qnext;         // 8 queue heads kQueueStride apart, zeroed by the reduce pass
    const int* __restrict__ qbound;  // [9]: queue k holds tiles [qbound[k], qbound[k+1])
    const int2* __restrict__ lblk;   // (instance, link block)
    const int* __restrict__ nlblk;   // number of link blocks
    int ninst;                       // instance slots
    int tile_h;
    int persistent;                  // 1: tile queues, 0: one workgroup per tile
};

// Tables that a launch only reads (the instance descriptors, states, tile
// and link-block lists: written by the host, or by earlier launches), read
// through the constant address space.  The compiler then loads them from a
// uniform address with scalar loads into scalar registers, as it does the
// kernel arguments; read through a generic pointer they come in as vector
// loads (the launch's own stores might alias them) and every use needs a
// v_readfirstlane.  The scalar cache is invalidated when a launch starts.
// (The host pass of the compiler, which only checks these functions, has no
// such address space.)
#if defined(__HIP_DEVICE_COMPILE__)
#define LBM_CONST_AS __attribute__((address_space(4)))
#else
#define LBM_CONST_AS
#endif
template <typename T>
__device__ __forceinline__ const LBM_CONST_AS T* ro(const T* p) {
    return (const LBM_CONST_AS T*)p;
}

template <typename S, typename I_t>
__device__ __forceinline__ MainArgs<S> inst_main_args(const I_t& I, long long t, int tile_h) {
    MainArgs<S> a;
    const int c = int(t & 1);
    a.src = static_cast<const S*>(I.f[c]);
    a.dst = static_cast<S*>(I.f[c ^ 1]);
    a.flags = I.flags;
    a.side_idx = I.side_idx;
    a.psiw = I.psiw;
    a.side_mom = I.side_mom;
    a.side_f = I.side_f;
    a.partial = I.partial;
    a.mom_out = nullptr;
    a.nx = I.nx;
    a.ny = I.ny;
    a.pitch = I.pitch;
    a.plane = I.plane;
    a.tile_h = tile_h;
    a.nsegs = I.nsegs;
    a.nstrips = I.nstrips;
    a.side_mom_bytes = I.side_mom_bytes;
    a.side_f_bytes = I.side_f_bytes;
    return a;
}

template <typename S, typename R, int EOS, int DEV, bool SAVEF, int RING>
__device__ __forceinline__ void batch_tile(const BatchArgs& b, int g) {
    g = __builtin_amdgcn_readfirstlane(g);
    const int2 te = ro(b.tiles)[g];
    const BState st = ro<BState>(b.state)[te.x];
    if (st.remaining <= 0) return;
    const auto& I = ro(b.inst)[te.x];
    const Phys<double> ph = I.ph;
    main_tile<S, R, EOS, false, DEV, SAVEF, RING>(inst_main_args<S>(I, st.t, b.tile_h),
                                                  phys_as<R>(ph), te.y);
}

// Persistent form: a fixed grid; each workgroup takes tiles from the queue
// of its XCD (workgroups are dispatched to the XCDs round robin), then from
// the other queues in turn, until all are empty.  The queues hold
// contiguous runs of the tile list, so one XCD works through compact
// pieces of the same instances and finds their halos in its L2.
template <typename S, typename R, int EOS, int DEV, bool SAVEF, int RING>
// (at least three wavefronts per SIMD: a ring of four rows would otherwise
// take more registers than three leave)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_main_batch(
    BatchArgs b) {
    if (!b.persistent) {
        batch_tile<S, R, EOS, DEV, SAVEF, RING>(b, xcd_tile(blockIdx.x, gridDim.x));
        return;
    }
    __shared__ int s_g;
    const int xcd = blockIdx.x & 7;
    int qi = 0;
    for (;;) {
        __syncthreads();  // the previous tile is done with s_g and the LDS ring
        if (threadIdx.x == 0) {
            int g = -1;
            while (qi < 8) {
                const int q = (xcd + qi) & 7;
                const int k = b.qbound[q] + atomicAdd(&b.qnext[q * kQueueStride], 1);
                if (k < b.qbound[q + 1]) {
                    g = k;
                    break;
                }
                ++qi;
            }
            s_g = g;
        }
        __syncthreads();
        const int g = s_g;
        if (g < 0) break;
        batch_tile<S, R, EOS, DEV, SAVEF, RING>(b, g);
    }
}

template <typename S, int DEV>
__global__ __launch_bounds__(256) void k_boundary_batch(BatchArgs b) {
    const int n = *ro(b.nlblk);
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        const int2 e = ro(b.lblk)[k];
        const BState st = ro<BState>(b.state)[e.x];
        if (st.remaining <= 0) continue;
        const auto& I = ro(b.inst)[e.x];
        BndArgs a;
        a.nslot = I.nslot;
        a.lnode = I.lnode;
        a.lmeta = I.lmeta;
        a.lghost = I.lghost;
        a.lxf = I.lxf;
        a.lxff = I.lxff;
        a.lslotb = I.lslotb;
        a.lslotf = I.lslotf;
        a.lc = I.lc;
        a.luw = I.luw;
        a.side_mom = I.side_mom;
        a.side_f = I.side_f;
        a.plane = I.plane;
        a.rref = I.rref;
        a.lref = I.lref;
        a.fix = I.fix;
        a.partial = nullptr;
        a.partial2 = nullptr;
        a.np = 0;
        a.hist = nullptr;
        a.cap = 1;
        a.clock = nullptr;
        a.unstable = nullptr;
        a.do_reduce = 0;
        a.force = nullptr;
        a.negrest = nullptr;
        a.degen = nullptr;
        a.nlink_blocks = 0;
        a.open_x = 0;
        a.nx = a.ny = a.pitch = 0;
        a.inlet_u = 0.0;
        __syncthreads();  // the previous block is done with the LDS
        boundary_block<S, DEV>(static_cast<S*>(I.f[st.t & 1]), a, e.y);
    }
}

// Per instance: M(t+1) from the main pass's partials in a fixed order, the
// first non-finite mass, t += 1 and one step fewer to run (none once
// unstable).  Also empties the tile queues for the next main pass.
template <int Unused = 0>
__global__ __launch_bounds__(256) void k_reduce_batch(BatchArgs b) {
    for (int i = blockIdx.x; i < b.ninst; i += gridDim.x) {
        BState* st = b.state + i;
        const long long rem = st->remaining;
        if (rem <= 0) continue;
        const auto& I = ro(b.inst)[i];
        const long long t1 = st->t + 1;
        __syncthreads();
        reduce_partials(I.partial, I.np, I.hist, t1 % I.cap, t1, I.unstable);
        if (threadIdx.x == 0) {
            st->t = t1;
            st->remaining = *I.unstable >= 0 ? 0 : rem - 1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < 8) b.qnext[threadIdx.x * kQueueStride] = 0;
}

}  // namespace lbm
