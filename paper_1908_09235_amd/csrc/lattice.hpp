// D2Q9 lattice, equation of state, equilibrium, forcing and collision for
// the device.  Directions: 0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0), 4 (0,-1),
// 5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1).
//
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
    R e0, e1, e2, e3;  // EOS parameters
    R p2G;             // 2 / G
    R rref;            // reference density of deviation storage (else 0)
    R s[9];        // relaxation rates of the nine moments (BGK: all 1/tau)
    R h[9];        // 1 - s/2: the weight of the forcing source per moment
};

template <typename R>
__host__ __device__ __forceinline__ Phys<R> phys_as(const Phys<double>& d) {
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
    for (int i = 0; i < 9; ++i) p.h[i] = R(d.h[i]);
    return p;
}

enum { EOS_NONE = 0, EOS_EXP = 1, EOS_CS = 2 };

// Reciprocal and square root.  FP64 reciprocal: the hardware estimate
// refined by two Newton steps r <- r + r (1 - x r), within an ulp (the
// argument is a density or a positive power of one); FP64 square root
// correctly rounded; FP32: the hardware instructions (1 ulp).  On the host,
// plain division and square root.
__host__ __device__ __forceinline__ double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ double root(double x) { return sqrt(x); }
__host__ __device__ __forceinline__ float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float root(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// Pseudopotential.  EXP: psi0 exp(-rho0/rho).  CS: sqrt(2 (p - rho/3)/G)
// with p the Carnahan-Starling pressure.  p2G = 2/G.
template <int EOS, typename R>
__host__ __device__ __forceinline__ R psi_of(R rho, const Phys<R>& p) {
    if constexpr (EOS == EOS_EXP) {
        return p.e0 * exp(-p.e1 * rcp(rho));
    } else if constexpr (EOS == EOS_CS) {
        const R a = p.e0, b = p.e1, Rg = p.e2, T = p.e3;
        const R eta = R(0.25) * b * rho;
        const R num = fma(eta, fma(eta, R(1) - eta, R(1)), R(1));
        const R om = R(1) - eta;
        const R den = om * om * om;
        const R pe = fma(-a * rho, rho, (rho * Rg * T) * num * rcp(den));
        return root(p.p2G * fma(rho, R(-1.0 / 3.0), pe));
    } else {
        return R(0);
    }
}

// Collision, Eq. (2), with Guo forcing, in the D2Q9 moment space of
// Lallemand & Luo (rows rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy):
//   m* = m + S (m_eq - m) + (I - S/2) M Fbar,   f* = f + M^-1 (m* - m).
// BGK is the case of equal rates 1/tau.  The equilibrium moments of Eq. (4)
// and the moments of the Guo source are written in closed form:
//   e_eq = -2 rho + 3 rho u^2, eps_eq = rho - 3 rho u^2, j = rho u,
//   q_eq = -rho u, p_xx,eq = rho (ux^2 - uy^2), p_xy,eq = rho ux uy;
//   (M Fbar) = (0, 6 u.F, -6 u.F, Fx, -Fx, Fy, -Fy, 2 (ux Fx - uy Fy),
//               ux Fy + uy Fx).
// With j_eq - j = F/2 (Eq. 5) the momentum moments change by exactly F.
// The update is formed as increments of the populations, opposite
// directions paired, and the rest increment closes the mass balance, so
// the arithmetic acts on the small non-equilibrium parts and each
// expression is exactly symmetric under lattice reflections.
//
// h holds the populations in their stored form: f itself, or the deviations
// g = f - w rho_ref; drho = sum h (= rho - rho_ref).  The lattice weights
// have e- and eps-moments -2 and 1 and no others, so only those two moments
// see the reference.  The increments are returned in dh.
template <typename R>
__device__ __forceinline__ void collide(const R f[9], R rho, R drho, R ux, R uy, R Fx,
                                        R Fy, const Phys<R>& p, R dh[9]) {
    const R s1 = f[1] + f[3], s2 = f[2] + f[4], c1 = f[5] + f[7], c2 = f[6] + f[8];
    const R d1 = f[1] - f[3], d2 = f[2] - f[4], e1 = f[5] - f[7], e2 = f[6] - f[8];
    const R sa = s1 + s2, sd = c1 + c2;
    const R m_e = fma(R(-4), f[0], (sd + sd) - sa);
    const R m_p = fma(R(4), f[0], sd - (sa + sa));
    const R m_qx = (e1 - e2) - (d1 + d1);
    const R m_qy = (e1 + e2) - (d2 + d2);
    const R m_xx = s1 - s2, m_xy = c1 - c2;
    const R uxx = ux * ux, uyy = uy * uy, usq = uxx + uyy;
    const R uF6 = R(6) * fma(ux, Fx, uy * Fy);
    const R ru2 = R(3) * rho * usq;
    // h = 1 - s/2 weighs the source moments; multiply-adds written out
    const R De = fma(p.s[1], (ru2 - (drho + drho)) - m_e, p.h[1] * uF6);
    const R Dp = fma(p.s[2], (drho - ru2) - m_p, -p.h[2] * uF6);
    const R Dqx = fma(-p.s[4], fma(rho, ux, m_qx), -p.h[4] * Fx);
    const R Dqy = fma(-p.s[6], fma(rho, uy, m_qy), -p.h[6] * Fy);
    const R Dxx = fma(p.s[7], fma(rho, uxx - uyy, -m_xx), p.h[7] * (R(2) * fma(ux, Fx, -uy * Fy)));
    const R Dxy = fma(p.s[8], fma(rho, ux * uy, -m_xy), p.h[8] * fma(ux, Fy, uy * Fx));
    // M^-1 = M^T diag(1/|row|^2), |row|^2 = 9, 36, 36, 6, 12, 6, 12, 4, 4
    const R kjx = Fx * R(1.0 / 6.0), kjy = Fy * R(1.0 / 6.0);
    const R kxx = Dxx * R(0.25), kxy = Dxy * R(0.25);
    const R A = fma(Dp, R(-2.0 / 36.0), De * R(-1.0 / 36.0));
    const R B = fma(De, R(2.0 / 36.0), Dp * R(1.0 / 36.0));
    const R X = fma(Dqx, R(-2.0 / 12.0), kjx), Y = fma(Dqy, R(-2.0 / 12.0), kjy);
    const R P = fma(Dqx, R(1.0 / 12.0), kjx), Q = fma(Dqy, R(1.0 / 12.0), kjy);
    const R g1 = (A + kxx) + X, g3 = (A + kxx) - X;
    const R g2 = (A - kxx) + Y, g4 = (A - kxx) - Y;
    const R bp = B + kxy, bm = B - kxy;
    const R g5 = bp + (P + Q), g7 = bp - (P + Q);
    const R g6 = bm + (Q - P), g8 = bm - (Q - P);
    const R g0 = -(((g1 + g3) + (g2 + g4)) + ((g5 + g7) + (g6 + g8)));
    dh[0] = g0;
    dh[1] = g1;
    dh[2] = g2;
    dh[3] = g3;
    dh[4] = g4;
    dh[5] = g5;
    dh[6] = g6;
    dh[7] = g7;
    dh[8] = g8;
}

}  // namespace lbm
