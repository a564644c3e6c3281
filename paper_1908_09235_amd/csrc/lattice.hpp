// D2Q9 lattice, equation of state, equilibrium, forcing and collision for
// the device.  Directions: 0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
// 5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1).
//
// Products with the lattice velocity components (0, +1, -1) are written as
// the signed sums they are, so that each expression rounds exactly as the
// textbook formula evaluated left to right.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

__host__ __device__ constexpr int cx(int a) {
    return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int a) {
    return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int a) {
    return a == 0 ? 0 : (a <= 4 ? ((a + 1) & 3) + 1 : ((a - 5 + 2) & 3) + 5);
}
// lattice weights of Eq. (4)
__host__ __device__ constexpr double wt(int a) {
    return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// interaction weights of Eq. (16)
__host__ __device__ constexpr double wf(int a) {
    return a == 0 ? 0.0 : (a <= 4 ? 1.0 / 3.0 : 1.0 / 12.0);
}

// e_a . v, exact
template <typename R>
__host__ __device__ __forceinline__ R edot(int a, R vx, R vy) {
    switch (a) {
    case 1: return vx;
    case 2: return vy;
    case 3: return -vx;
    case 4: return -vy;
    case 5: return vx + vy;
    case 6: return -vx + vy;
    case 7: return -vx - vy;
    case 8: return vx - vy;
    default: return R(0);
    }
}

// physical parameters, in the compute type
template <typename R>
struct Phys {
    R G, gx, gy;
    R omega;       // 1/tau
    R guo_pref;    // 1 - 1/(2 tau)
    R e0, e1, e2, e3;  // EOS parameters
    R s[9];        // MRT rates
};

enum { EOS_NONE = 0, EOS_EXP = 1, EOS_CS = 2 };
enum { COLL_BGK = 0, COLL_MRT = 1 };

// Pseudopotential.  EXP: psi0 exp(-rho0/rho).  CS: sqrt(2 (p - rho/3)/G)
// with p the Carnahan-Starling pressure.
template <int EOS, typename R>
__host__ __device__ __forceinline__ R psi_of(R rho, const Phys<R>& p) {
    if constexpr (EOS == EOS_EXP) {
        return p.e0 * exp(-p.e1 / rho);
    } else if constexpr (EOS == EOS_CS) {
        const R a = p.e0, b = p.e1, Rg = p.e2, T = p.e3;
        const R eta = b * rho / R(4);
        const R num = R(1) + eta + eta * eta - eta * eta * eta;
        const R den = (R(1) - eta) * (R(1) - eta) * (R(1) - eta);
        const R pe = rho * Rg * T * num / den - a * rho * rho;
        const R v = R(2) * (pe - rho * R(1.0 / 3.0)) / p.G;
        return sqrt(v);
    } else {
        return R(0);
    }
}

// Equilibrium, Eq. (4): w rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u)
template <typename R>
__device__ __forceinline__ R feq_a(int a, R rho, R ux, R uy, R usq) {
    const R eu = edot<R>(a, ux, uy);
    return R(wt(a)) * rho * (R(1) + R(3) * eu + R(4.5) * (eu * eu) - R(1.5) * usq);
}

// Guo source without its prefactor: w [3 (e - u) + 9 (e.u) e] . F
template <typename R>
__device__ __forceinline__ R guo_raw_a(int a, R ux, R uy, R Fx, R Fy) {
    const R eu = edot<R>(a, ux, uy);
    R gx = R(3) * (R(cx(a)) - ux);
    R gy = R(3) * (R(cy(a)) - uy);
    if (cx(a) == 1) gx = gx + R(9) * eu;
    if (cx(a) == -1) gx = gx + -(R(9) * eu);
    if (cy(a) == 1) gy = gy + R(9) * eu;
    if (cy(a) == -1) gy = gy + -(R(9) * eu);
    return gx * Fx + gy * Fy;
}

// Lallemand-Luo D2Q9 moment basis: integer matrix entries.
__host__ __device__ constexpr int mrt_m(int i, int a) {
    // rows: rho, e, eps, jx, qx, jy, qy, pxx, pxy
    return i == 0 ? 1
         : i == 1 ? (a == 0 ? -4 : (a <= 4 ? -1 : 2))
         : i == 2 ? (a == 0 ? 4 : (a <= 4 ? -2 : 1))
         : i == 3 ? cx(a)
         : i == 4 ? (a == 0 ? 0 : (a <= 4 ? -2 * cx(a) : cx(a)))
         : i == 5 ? cy(a)
         : i == 6 ? (a == 0 ? 0 : (a <= 4 ? -2 * cy(a) : cy(a)))
         : i == 7 ? cx(a) * cx(a) - cy(a) * cy(a)
         : cx(a) * cy(a);
}
__host__ __device__ constexpr int mrt_norm2(int i) {
    return i == 0 ? 9 : i == 1 ? 36 : i == 2 ? 36 : i == 3 ? 6 : i == 4 ? 12
         : i == 5 ? 6 : i == 6 ? 12 : 4;
}

// y = M x, summed in direction order (zero entries skipped: adding a signed
// zero never changes a sum)
template <typename R>
__device__ __forceinline__ void mrt_fwd(const R x[9], R y[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        R acc = R(0);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int m = mrt_m(i, a);
            if (m == 1) acc = acc + x[a];
            else if (m == -1) acc = acc + -x[a];
            else if (m != 0) acc = acc + R(m) * x[a];
        }
        y[i] = acc;
    }
}

// x = M^-1 y with M^-1 = M^T diag(1/|row|^2)
template <typename R>
__device__ __forceinline__ void mrt_inv(const R y[9], R x[9]) {
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        R acc = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int m = mrt_m(i, a);
            if (m != 0) acc = acc + R(double(m) / double(mrt_norm2(i))) * y[i];
        }
        x[a] = acc;
    }
}

// Collision, Eq. (2), with Guo forcing.  f is overwritten by f*.
//
// In FP32 the rounded lattice weights sum to 1 + 7e-9, so the textbook form
// would create that much mass at every collision; there the rest population
// is taken from mass conservation instead, f*_0 = rho - sum_{a>0} f*_a,
// which is the same value in exact arithmetic.
template <int COLL, typename R>
__device__ __forceinline__ void collide(R f[9], R rho, R ux, R uy, R Fx, R Fy,
                                        const Phys<R>& p) {
    constexpr bool kMassExact = sizeof(R) == 4;
    const R usq = ux * ux + uy * uy;
    if constexpr (COLL == COLL_BGK) {
#pragma unroll
        for (int a = kMassExact ? 1 : 0; a < 9; ++a) {
            const R feq = feq_a<R>(a, rho, ux, uy, usq);
            const R guo = p.guo_pref * R(wt(a)) * guo_raw_a<R>(a, ux, uy, Fx, Fy);
            f[a] = f[a] - p.omega * (f[a] - feq) + guo;
        }
        if constexpr (kMassExact)
            f[0] = rho - (f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
    } else {
        R feq[9], fb[9], m[9], meq[9], mf[9], ms[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            feq[a] = feq_a<R>(a, rho, ux, uy, usq);
            fb[a] = R(wt(a)) * guo_raw_a<R>(a, ux, uy, Fx, Fy);
        }
        mrt_fwd<R>(f, m);
        mrt_fwd<R>(feq, meq);
        mrt_fwd<R>(fb, mf);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            ms[i] = m[i] - p.s[i] * (m[i] - meq[i]) + (R(1) - p.s[i] / R(2)) * mf[i];
        mrt_inv<R>(ms, f);
        if constexpr (kMassExact)
            f[0] = rho - (f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]);
    }
}

}  // namespace lbm
