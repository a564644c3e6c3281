/*
 * Plain FP64 CPU oracle: the two-phase D2Q9 lattice-Boltzmann step of
 * Yu, Li & Wen (arXiv:1908.09235), written as a slow, textbook sequence.
 *
 * TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).  No blocking, no fusion, no
 * ghost slots: every step of the method is its own loop over the lattice, in
 * the order the paper states it:
 *   1. density, Eq. (5)
 *   2. pseudopotential psi(rho); solid nodes carry a constant virtual wall
 *      value (contact-angle treatment, Sec. 3.2)
 *   3. interaction force, Eq. (16), plus a body force rho*g (Sec. 3.1)
 *   4. velocity with the half-force shift, Eq. (5)
 *   5. collision, Eq. (2), with the equilibrium of Eq. (4) and the forcing
 *      term of Guo et al. (2002), which the paper cites (Sec. 3.2); or the
 *      D2Q9 multiple-relaxation-time form of the same step
 *   6. streaming, Eq. (3); with open x boundaries, the populations that
 *      enter from outside: Zou-He velocity inlet at x = 0, fully developed
 *      (zero-gradient) outlet at x = nx - 1 (Sec. 4.2)
 *   7. one curved-wall rule per cut link, Eqs. (7)-(14), and the force on
 *      the walls by momentum exchange (Sec. 4.2)
 *   8. per boundary node: the leak of Eq. (15) and the corrections of
 *      scheme A (Eq. 18), scheme B (Eqs. 20-22) or Bao et al. (Eq. 23)
 *   9. total mass, compensated (Neumaier) summation
 * Compiled with -ffp-contract=off so that every product and sum rounds as
 * written.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D2Q9 velocities and weights (Sec. 2.1, text under Eq. 4). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* Interaction weights of Eq. (16): 1/3 on axes, 1/12 on diagonals. */
static const double WF[9] = {0.0,        1.0 / 3.0,  1.0 / 3.0,
                             1.0 / 3.0,  1.0 / 3.0,  1.0 / 12.0,
                             1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};
/* c_s = 1/sqrt(3): 1/c_s^2 = 3, 1/(2 c_s^4) = 4.5, 1/(2 c_s^2) = 1.5 and
 * 1/c_s^4 = 9, all exact in binary floating point. */
static const double CS2 = 1.0 / 3.0;
static const double INV_CS2 = 3.0;
static const double INV_2CS4 = 4.5;
static const double INV_2CS2 = 1.5;
static const double INV_CS4 = 9.0;

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* ------------------------------------------------------------------ */
/* Equilibrium, Eq. (4):                                               */
/* f_eq = w rho [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)]       */
void ora_feq(double rho, double ux, double uy, double out[9]) {
    double usq = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        out[a] = WT[a] * rho *
                 (1.0 + INV_CS2 * eu + INV_2CS4 * (eu * eu) - INV_2CS2 * usq);
    }
}

/* Forcing term of Guo, Zheng & Shi (2002), cited in Sec. 3.2:          */
/* F_a = (1 - 1/(2 tau)) w_a [ (e_a - u)/cs^2 + (e_a.u) e_a / cs^4 ].F  */
void ora_guo(double tau, double ux, double uy, double Fx, double Fy,
             double out[9]) {
    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int a = 0; a < 9; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        double cx = INV_CS2 * (EX[a] - ux) + INV_CS4 * eu * EX[a];
        double cy = INV_CS2 * (EY[a] - uy) + INV_CS4 * eu * EY[a];
        out[a] = pref * WT[a] * (cx * Fx + cy * Fy);
    }
}

/* D2Q9 moment basis of Lallemand & Luo (2000), rows in the order
 * rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy, each built from its
 * polynomial in the lattice velocity c:
 *   e = -4 + 3|c|^2, eps = 4 - 21|c|^2/2 + 9|c|^4/2,
 *   q = (-5 + 3|c|^2) c, p_xx = cx^2 - cy^2, p_xy = cx cy.
 * The rows are orthogonal, so M^-1 = M^T diag(1/|row|^2). */
void ora_mrt_matrix(double M[81], double Minv[81]) {
    for (int a = 0; a < 9; ++a) {
        double cx = EX[a], cy = EY[a], c2 = cx * cx + cy * cy;
        M[0 * 9 + a] = 1.0;
        M[1 * 9 + a] = -4.0 + 3.0 * c2;
        M[2 * 9 + a] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
        M[3 * 9 + a] = cx;
        M[4 * 9 + a] = (-5.0 + 3.0 * c2) * cx;
        M[5 * 9 + a] = cy;
        M[6 * 9 + a] = (-5.0 + 3.0 * c2) * cy;
        M[7 * 9 + a] = cx * cx - cy * cy;
        M[8 * 9 + a] = cx * cy;
    }
    for (int i = 0; i < 9; ++i) {
        double n2 = 0.0;
        for (int a = 0; a < 9; ++a) n2 += M[i * 9 + a] * M[i * 9 + a];
        for (int a = 0; a < 9; ++a) Minv[a * 9 + i] = M[i * 9 + a] / n2;
    }
}

/* Collision, Eq. (2).  BGK: f* = f - (f - f_eq)/tau + F_a.
 * MRT: m* = m - S(m - m_eq) + (I - S/2) M Fbar, with m = M f,
 * m_eq = M f_eq and Fbar the Guo source without its (1 - 1/2tau)
 * prefactor; f* = M^-1 m*.  With every rate equal to 1/tau the MRT form
 * is the BGK form. */
void ora_collide(int32_t collision, double tau, const double s[9],
                 const double f[9], double rho, double ux, double uy,
                 double Fx, double Fy, double out[9]) {
    double feq[9];
    ora_feq(rho, ux, uy, feq);
    if (collision == ORA_COLL_BGK) {
        double guo[9];
        ora_guo(tau, ux, uy, Fx, Fy, guo);
        for (int a = 0; a < 9; ++a)
            out[a] = f[a] - (1.0 / tau) * (f[a] - feq[a]) + guo[a];
        return;
    }
    double M[81], Minv[81];
    ora_mrt_matrix(M, Minv);
    /* Guo source without its (1 - 1/(2 tau)) prefactor */
    double fbar[9];
    for (int a = 0; a < 9; ++a) {
        double eu = EX[a] * ux + EY[a] * uy;
        double cx = INV_CS2 * (EX[a] - ux) + INV_CS4 * eu * EX[a];
        double cy = INV_CS2 * (EY[a] - uy) + INV_CS4 * eu * EY[a];
        fbar[a] = WT[a] * (cx * Fx + cy * Fy);
    }
    double m[9], meq[9], mf[9], ms[9];
    for (int i = 0; i < 9; ++i) {
        m[i] = 0.0;
        meq[i] = 0.0;
        mf[i] = 0.0;
        for (int a = 0; a < 9; ++a) {
            m[i] += M[i * 9 + a] * f[a];
            meq[i] += M[i * 9 + a] * feq[a];
            mf[i] += M[i * 9 + a] * fbar[a];
        }
    }
    for (int i = 0; i < 9; ++i)
        ms[i] = m[i] - s[i] * (m[i] - meq[i]) + (1.0 - s[i] / 2.0) * mf[i];
    for (int a = 0; a < 9; ++a) {
        out[a] = 0.0;
        for (int i = 0; i < 9; ++i) out[a] += Minv[a * 9 + i] * ms[i];
    }
}

/* Equation-of-state pressure.  CS: Carnahan-Starling,
 * p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2,
 * eta = b rho / 4.  EXP: the pressure implied by psi, rho cs^2 + G psi^2/2
 * (needs G, so it is not defined here and returns NaN). */
double ora_pressure_eos(int32_t eos, const double p[4], double rho) {
    if (eos == ORA_EOS_CS) {
        double a = p[0], b = p[1], R = p[2], T = p[3];
        double eta = b * rho / 4.0;
        double num = 1.0 + eta + eta * eta - eta * eta * eta;
        double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
        return rho * R * T * num / den - a * rho * rho;
    }
    if (eos == ORA_EOS_NONE) return rho * CS2;
    return NAN;
}

/* Pseudopotential.  EXP (Sec. 3.2): psi = psi0 exp(-rho0/rho).
 * CS: psi = sqrt(2 (p_EOS - rho cs^2) / G), so that the model pressure
 * rho cs^2 + G psi^2 / 2 equals the equation of state.  NONE: no
 * interaction. */
double ora_psi(int32_t eos, const double p[4], double G, double rho) {
    if (eos == ORA_EOS_EXP) return p[0] * exp(-p[1] / rho);
    if (eos == ORA_EOS_CS) {
        double pe = ora_pressure_eos(eos, p, rho);
        double v = 2.0 * (pe - rho * CS2) / G;
        return sqrt(v); /* NaN when v < 0: caught as non-finite mass */
    }
    return 0.0;
}

/* ------------------------------------------------------------------ */
/* One cut link (x_b, a, q): the incoming f_abar(x_b, t+1).             */
double ora_rule_incoming(int32_t rule, int32_t dir, double q, double tau,
                         const double in[15], double rho_eq,
                         double *chi_out, double *bracket_out) {
    const double fa_b = in[0], fab_b = in[1], fa_f = in[2], fab_f = in[3];
    const double fa_ff = in[4], fpre_a = in[5], rho_b = in[6];
    const double ubx = in[7], uby = in[8], ufx = in[9], ufy = in[10];
    const double uwx = in[11], uwy = in[12];
    const int f_ok = in[13] != 0.0, ff_ok = in[14] != 0.0;
    const double ex = EX[dir], ey = EY[dir];
    /* Momentum that a wall moving at u_w adds on reflection (Ladd; Mei et
     * al. 1999): 2 w_a rho_b (e_a.u_w)/cs^2.  Zero for the paper's walls. */
    const double wall = 2.0 * WT[dir] * rho_b * INV_CS2 * (ex * uwx + ey * uwy);
    double chi = 0.0, bracket = 0.0, result;

    switch (rule) {
    case ORA_RULE_HALFWAY:
        /* f_abar(x_b,t+1) = f*_a(x_b,t): the q = 1/2 limit (Sec. 2.2). */
        result = fa_b - wall;
        break;
    case ORA_RULE_FH:
    case ORA_RULE_MLS: {
        double usx, usy;
        if (q < 0.5) {
            if (rule == ORA_RULE_FH) {
                /* Eq. (9) */
                usx = ubx;
                usy = uby;
                chi = (2.0 * q - 1.0) / (tau - 1.0);
            } else {
                /* Eq. (11); x_f solid: use u_b instead of u_f */
                usx = f_ok ? ufx : ubx;
                usy = f_ok ? ufy : uby;
                chi = (2.0 * q - 1.0) / (tau - 2.0);
            }
        } else {
            /* Eq. (10) */
            usx = (q - 1.0) / q * ubx + uwx / q;
            usy = (q - 1.0) / q * uby + uwy / q;
            chi = (2.0 * q - 1.0) / tau;
        }
        /* Eq. (8) / Eq. (20): w_a rho [1 + e.u_s/cs^2 + (e.u_b)^2/(2cs^4)
         * - u_b.u_b/(2 cs^2)] */
        double eus = ex * usx + ey * usy;
        double eub = ex * ubx + ey * uby;
        double ub2 = ubx * ubx + uby * uby;
        bracket = WT[dir] * (1.0 + INV_CS2 * eus + INV_2CS4 * (eub * eub) -
                             INV_2CS2 * ub2);
        double feq_s = rho_eq * bracket;
        /* Eq. (7) with f_abar(x_b,t+1) = f*_abar(x_s,t) */
        result = (1.0 - chi) * fa_b + chi * feq_s - wall;
        break;
    }
    case ORA_RULE_IBB_LINEAR:
        /* Eq. (12); q < 1/2 with x_f solid falls back to the other branch */
        if (q < 0.5 && f_ok)
            result = 2.0 * q * fa_b + (1.0 - 2.0 * q) * fa_f;
        else
            result = 1.0 / (2.0 * q) * fa_b + (2.0 * q - 1.0) / (2.0 * q) * fab_b;
        break;
    case ORA_RULE_IBB_QUADRATIC:
        /* Eq. (13); a missing x_f or x_ff falls back to Eq. (12) */
        if (q < 0.5 && f_ok && ff_ok)
            result = q * (1.0 + 2.0 * q) * fa_b + (1.0 - 4.0 * q * q) * fa_f -
                     q * (1.0 - 2.0 * q) * fa_ff;
        else if (q >= 0.5 && f_ok)
            result = 1.0 / (q * (2.0 * q + 1.0)) * fa_b +
                     (2.0 * q - 1.0) / q * fab_b -
                     (2.0 * q - 1.0) / (2.0 * q + 1.0) * fab_f;
        else if (q < 0.5 && f_ok)
            result = 2.0 * q * fa_b + (1.0 - 2.0 * q) * fa_f;
        else
            result = 1.0 / (2.0 * q) * fa_b + (2.0 * q - 1.0) / (2.0 * q) * fab_b;
        break;
    case ORA_RULE_ZHAO_YONG:
        /* Eq. (14): post-collision f*_abar and pre-collision f_a at x_b */
        result = 2.0 * q / (1.0 + 2.0 * q) * fab_b + 1.0 / (1.0 + 2.0 * q) * fpre_a;
        break;
    default:
        result = NAN;
    }
    if (chi_out) *chi_out = chi;
    if (bracket_out) *bracket_out = bracket;
    return result;
}

/* ------------------------------------------------------------------ */
struct ora_sim {
    int nx, ny;
    int64_t N;
    uint8_t *solid;
    double *psiw;
    int32_t eos, collision, rule, fix;
    double eos_p[4], G, gx, gy, tau, s[9];
    double *f, *fs, *fn;            /* [9][N]                           */
    double *rho, *ux, *uy, *psi, *Fx, *Fy;
    int64_t nlinks;
    int32_t *lx, *ly, *ldir;        /* sorted by node index, then dir   */
    double *lq, *luwx, *luwy;
    int64_t nb;                     /* boundary nodes                   */
    int64_t *bstart, *bnode;        /* CSR over links                   */
    double *leaks;
    int64_t counters[5];
    int64_t t;
    int32_t open_x;
    double inlet_u;
    double force[2];
};

static void free_sim(ora_sim *s) {
    if (!s) return;
    free(s->solid); free(s->psiw); free(s->f); free(s->fs); free(s->fn);
    free(s->rho); free(s->ux); free(s->uy); free(s->psi); free(s->Fx);
    free(s->Fy); free(s->lx); free(s->ly); free(s->ldir); free(s->lq);
    free(s->luwx); free(s->luwy); free(s->bstart); free(s->bnode);
    free(s->leaks);
    free(s);
}

void ora_destroy(ora_sim *s) { free_sim(s); }

typedef struct { int64_t node; int32_t dir; int64_t src; } link_key;

static int cmp_key(const void *pa, const void *pb) {
    const link_key *a = (const link_key *)pa, *b = (const link_key *)pb;
    if (a->node != b->node) return a->node < b->node ? -1 : 1;
    return a->dir - b->dir;
}

int ora_create(const ora_desc *d, ora_sim **out) {
    if (!d || !out || d->nx < 3 || d->ny < 3 || !d->solid || !d->rho0)
        return -1;
    if (!(d->tau > 0.5) || !isfinite(d->tau)) return -1;
    if (d->rule < 0 || d->rule > 5 || d->fix < 0 || d->fix > 3) return -1;
    if (d->eos < 0 || d->eos > 2 || d->collision < 0 || d->collision > 1)
        return -1;
    if ((d->fix == ORA_FIX_B || d->fix == ORA_FIX_BAO) &&
        d->rule != ORA_RULE_FH && d->rule != ORA_RULE_MLS)
        return -1;
    if (d->eos != ORA_EOS_NONE && (d->G == 0.0 || !isfinite(d->G))) return -1;
    if (d->collision == ORA_COLL_MRT) {
        for (int i = 0; i < 9; ++i)
            if (!(d->mrt_s[i] > 0.0 && d->mrt_s[i] < 2.0)) return -1;
        if (fabs(d->mrt_s[7] - 1.0 / d->tau) > 1e-12 ||
            fabs(d->mrt_s[8] - 1.0 / d->tau) > 1e-12)
            return -1;
    }
    if (d->open_x != 0 && d->open_x != 1) return -1;
    if (d->open_x) {
        /* single phase only; the inlet density formula needs |U| < 1; the
         * three outermost columns on each side are fluid, so that no wall
         * rule reaches across the seam (x_ff of a cut link stays inside) */
        if (d->eos != ORA_EOS_NONE || !(fabs(d->inlet_u) < 1.0) || d->nx < 8) return -1;
        for (int y = 0; y < d->ny; ++y)
            for (int x = 0; x < d->nx; ++x)
                if ((x < 3 || x >= d->nx - 3) && d->solid[(int64_t)y * d->nx + x]) return -1;
    }
    const int nx = d->nx, ny = d->ny;
    const int64_t N = (int64_t)nx * ny;
    ora_sim *s = (ora_sim *)calloc(1, sizeof(ora_sim));
    if (!s) return -1;
    s->nx = nx; s->ny = ny; s->N = N;
    s->eos = d->eos; s->collision = d->collision; s->rule = d->rule;
    s->fix = d->fix; s->G = d->G; s->gx = d->gx; s->gy = d->gy;
    s->tau = d->tau;
    memcpy(s->eos_p, d->eos_p, sizeof(s->eos_p));
    if (d->collision == ORA_COLL_MRT) memcpy(s->s, d->mrt_s, sizeof(s->s));
    s->solid = (uint8_t *)malloc(N);
    s->psiw = (double *)calloc(N, sizeof(double));
    s->f = (double *)calloc(9 * N, sizeof(double));
    s->fs = (double *)calloc(9 * N, sizeof(double));
    s->fn = (double *)calloc(9 * N, sizeof(double));
    s->rho = (double *)calloc(N, sizeof(double));
    s->ux = (double *)calloc(N, sizeof(double));
    s->uy = (double *)calloc(N, sizeof(double));
    s->psi = (double *)calloc(N, sizeof(double));
    s->Fx = (double *)calloc(N, sizeof(double));
    s->Fy = (double *)calloc(N, sizeof(double));
    if (!s->solid || !s->psiw || !s->f || !s->fs || !s->fn || !s->rho ||
        !s->ux || !s->uy || !s->psi || !s->Fx || !s->Fy) {
        free_sim(s);
        return -1;
    }
    for (int64_t i = 0; i < N; ++i) s->solid[i] = d->solid[i] ? 1 : 0;
    /* contact angle: solid nodes carry psi of a constant virtual wall
     * density (Sec. 3.2) */
    for (int64_t i = 0; i < N; ++i) {
        if (s->solid[i]) {
            double rw = d->rho_wall ? d->rho_wall[i] : 0.0;
            double v = (s->eos == ORA_EOS_NONE)
                           ? 0.0
                           : ora_psi(s->eos, s->eos_p, s->G, rw);
            if (!isfinite(v) || (s->eos != ORA_EOS_NONE && !(rw > 0.0))) {
                free_sim(s);
                return -1;
            }
            s->psiw[i] = v;
        }
    }
    /* links: validate, sort by (node, dir), detect duplicates */
    int64_t L = d->nlinks;
    if (L < 0 || (L > 0 && (!d->link_x || !d->link_y || !d->link_dir ||
                            !d->link_q))) {
        free_sim(s);
        return -1;
    }
    link_key *keys = (link_key *)malloc((L > 0 ? L : 1) * sizeof(link_key));
    if (!keys) { free_sim(s); return -1; }
    int bad = 0, singular = 0;
    for (int64_t k = 0; k < L; ++k) {
        int x = d->link_x[k], y = d->link_y[k], a = d->link_dir[k];
        double q = d->link_q[k];
        if (x < 0 || x >= nx || y < 0 || y >= ny || a < 1 || a > 8) { bad = 1; break; }
        int64_t b = (int64_t)y * nx + x;
        int64_t xs = (int64_t)wrap(y + EY[a], ny) * nx + wrap(x + EX[a], nx);
        if (s->solid[b] || !s->solid[xs]) { bad = 1; break; }
        if (!(q > 0.0 && q <= 1.0)) { bad = 1; break; }
        double uwx = d->link_uwx ? d->link_uwx[k] : 0.0;
        double uwy = d->link_uwy ? d->link_uwy[k] : 0.0;
        if (!isfinite(uwx) || !isfinite(uwy)) { bad = 1; break; }
        if ((uwx != 0.0 || uwy != 0.0) &&
            !(d->rule == ORA_RULE_HALFWAY || d->rule == ORA_RULE_FH ||
              d->rule == ORA_RULE_MLS) ) { bad = 1; break; }
        if ((uwx != 0.0 || uwy != 0.0) && d->fix == ORA_FIX_BAO) { bad = 1; break; }
        if (d->rule == ORA_RULE_FH && q < 0.5 && fabs(d->tau - 1.0) < 1e-12)
            singular = 1;
        keys[k].node = b;
        keys[k].dir = a;
        keys[k].src = k;
    }
    if (bad) { free(keys); free_sim(s); return -1; }
    if (singular) { free(keys); free_sim(s); return -4; }
    qsort(keys, (size_t)L, sizeof(link_key), cmp_key);
    for (int64_t k = 1; k < L; ++k)
        if (keys[k].node == keys[k - 1].node && keys[k].dir == keys[k - 1].dir) {
            free(keys); free_sim(s); return -1;
        }
    /* every fluid->solid adjacency must carry exactly one link */
    {
        int64_t count = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (s->solid[i]) continue;
            int x = (int)(i % nx), y = (int)(i / nx);
            for (int a = 1; a < 9; ++a) {
                int64_t j = (int64_t)wrap(y + EY[a], ny) * nx + wrap(x + EX[a], nx);
                if (s->solid[j]) ++count;
            }
        }
        if (count != L) { free(keys); free_sim(s); return -1; }
    }
    s->nlinks = L;
    s->lx = (int32_t *)malloc((L + 1) * sizeof(int32_t));
    s->ly = (int32_t *)malloc((L + 1) * sizeof(int32_t));
    s->ldir = (int32_t *)malloc((L + 1) * sizeof(int32_t));
    s->lq = (double *)malloc((L + 1) * sizeof(double));
    s->luwx = (double *)malloc((L + 1) * sizeof(double));
    s->luwy = (double *)malloc((L + 1) * sizeof(double));
    s->bstart = (int64_t *)malloc((L + 2) * sizeof(int64_t));
    s->bnode = (int64_t *)malloc((L + 1) * sizeof(int64_t));
    s->leaks = (double *)calloc(L + 1, sizeof(double));
    if (!s->lx || !s->ly || !s->ldir || !s->lq || !s->luwx || !s->luwy ||
        !s->bstart || !s->bnode || !s->leaks) {
        free(keys); free_sim(s); return -1;
    }
    s->nb = 0;
    for (int64_t k = 0; k < L; ++k) {
        int64_t src = keys[k].src;
        s->lx[k] = d->link_x[src];
        s->ly[k] = d->link_y[src];
        s->ldir[k] = d->link_dir[src];
        s->lq[k] = d->link_q[src];
        s->luwx[k] = d->link_uwx ? d->link_uwx[src] : 0.0;
        s->luwy[k] = d->link_uwy ? d->link_uwy[src] : 0.0;
        if (k == 0 || keys[k].node != keys[k - 1].node) {
            s->bstart[s->nb] = k;
            s->bnode[s->nb] = keys[k].node;
            s->nb++;
        }
    }
    s->bstart[s->nb] = L;
    free(keys);
    /* initial state: f(0) = f_eq(rho0, u0) on fluid nodes */
    for (int64_t i = 0; i < N; ++i) {
        if (s->solid[i]) continue;
        double r = d->rho0[i];
        double vx = d->ux0 ? d->ux0[i] : 0.0, vy = d->uy0 ? d->uy0[i] : 0.0;
        if (!(r > 0.0) || !isfinite(r) || !isfinite(vx) || !isfinite(vy)) {
            free_sim(s); return -1;
        }
        if (s->eos == ORA_EOS_CS) {
            double v = ora_psi(s->eos, s->eos_p, s->G, r);
            if (!isfinite(v)) { free_sim(s); return -1; }
        }
        double feq[9];
        ora_feq(r, vx, vy, feq);
        for (int a = 0; a < 9; ++a) s->f[a * N + i] = feq[a];
    }
    s->t = 0;
    s->open_x = d->open_x;
    s->inlet_u = d->inlet_u;
    *out = s;
    return 0;
}

/* Steps 1-4: rho, psi, F, u from the pre-collision populations. */
static void macroscopic(ora_sim *s) {
    const int nx = s->nx, ny = s->ny;
    const int64_t N = s->N;
    for (int64_t i = 0; i < N; ++i) {
        if (s->solid[i]) { s->rho[i] = 0.0; continue; }
        double r = 0.0;
        for (int a = 0; a < 9; ++a) r += s->f[a * N + i];
        s->rho[i] = r;
    }
    for (int64_t i = 0; i < N; ++i)
        s->psi[i] = s->solid[i] ? s->psiw[i]
                                : ora_psi(s->eos, s->eos_p, s->G, s->rho[i]);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int64_t i = (int64_t)y * nx + x;
            if (s->solid[i]) {
                s->Fx[i] = s->Fy[i] = s->ux[i] = s->uy[i] = 0.0;
                continue;
            }
            double sx = 0.0, sy = 0.0;
            for (int a = 1; a < 9; ++a) {
                int64_t j = (int64_t)wrap(y + EY[a], ny) * nx + wrap(x + EX[a], nx);
                sx += WF[a] * s->psi[j] * EX[a];
                sy += WF[a] * s->psi[j] * EY[a];
            }
            double fx = 0.0, fy = 0.0;
            if (s->eos != ORA_EOS_NONE) {
                fx = -s->G * s->psi[i] * sx;
                fy = -s->G * s->psi[i] * sy;
            }
            fx += s->rho[i] * s->gx;
            fy += s->rho[i] * s->gy;
            s->Fx[i] = fx;
            s->Fy[i] = fy;
            double mx = 0.0, my = 0.0;
            for (int a = 0; a < 9; ++a) {
                mx += s->f[a * N + i] * EX[a];
                my += s->f[a * N + i] * EY[a];
            }
            s->ux[i] = (mx + fx / 2.0) / s->rho[i];
            s->uy[i] = (my + fy / 2.0) / s->rho[i];
        }
}

static double neumaier_add(double sum, double v, double *c) {
    double t = sum + v;
    if (fabs(sum) >= fabs(v))
        *c += (sum - t) + v;
    else
        *c += (v - t) + sum;
    return t;
}

static int one_step(ora_sim *s, double *mass_out) {
    const int nx = s->nx, ny = s->ny;
    const int64_t N = s->N;
    macroscopic(s);
    /* 5. collision */
    for (int64_t i = 0; i < N; ++i) {
        if (s->solid[i]) {
            for (int a = 0; a < 9; ++a) s->fs[a * N + i] = 0.0;
            continue;
        }
        double fl[9], out[9];
        for (int a = 0; a < 9; ++a) fl[a] = s->f[a * N + i];
        ora_collide(s->collision, s->tau, s->s, fl, s->rho[i], s->ux[i],
                    s->uy[i], s->Fx[i], s->Fy[i], out);
        for (int a = 0; a < 9; ++a) s->fs[a * N + i] = out[a];
    }
    /* 6. streaming: f_a(x + e_a, t+1) = f*_a(x, t) between fluid nodes;
     * what would come out of a solid node is left for step 7. */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int64_t i = (int64_t)y * nx + x;
            for (int a = 0; a < 9; ++a) s->fn[a * N + i] = 0.0;
            if (s->solid[i]) continue;
            for (int a = 0; a < 9; ++a) {
                int64_t j = (int64_t)wrap(y - EY[a], ny) * nx + wrap(x - EX[a], nx);
                s->fn[a * N + i] = s->solid[j] ? NAN : s->fs[a * N + j];
            }
        }
    /* 6b. open x boundaries (Sec. 4.2) */
    if (s->open_x) {
        const double U = s->inlet_u;
        for (int y = 0; y < ny; ++y) {
            /* inlet, x = 0: Zou and He (1997) for u = (U, 0); f1, f5, f8
             * arrive from outside */
            int64_t i = (int64_t)y * nx;
            double *f = s->fn;
            double rho = (f[0 * N + i] + f[2 * N + i] + f[4 * N + i] +
                          2.0 * (f[3 * N + i] + f[6 * N + i] + f[7 * N + i])) /
                         (1.0 - U);
            f[1 * N + i] = f[3 * N + i] + 2.0 / 3.0 * rho * U;
            f[5 * N + i] = f[7 * N + i] - 0.5 * (f[2 * N + i] - f[4 * N + i]) +
                           1.0 / 6.0 * rho * U;
            f[8 * N + i] = f[6 * N + i] + 0.5 * (f[2 * N + i] - f[4 * N + i]) +
                           1.0 / 6.0 * rho * U;
            /* outlet, x = nx - 1: f3, f6, f7 arrive from outside; fully
             * developed flow copies them from x = nx - 2 */
            int64_t o = (int64_t)y * nx + nx - 1;
            f[3 * N + o] = f[3 * N + o - 1];
            f[6 * N + o] = f[6 * N + o - 1];
            f[7 * N + o] = f[7 * N + o - 1];
        }
    }
    /* 7-8. cut links, leak and correction, node by node */
    s->force[0] = s->force[1] = 0.0;
    for (int64_t bi = 0; bi < s->nb; ++bi) {
        int64_t b = s->bnode[bi];
        int bx = (int)(b % nx), by = (int)(b / nx);
        int64_t k0 = s->bstart[bi], k1 = s->bstart[bi + 1];
        double in[8][15], inc[8], chi[8], br[8], wall[8];
        int dirs[8];
        int n = (int)(k1 - k0);
        for (int m = 0; m < n; ++m) {
            int64_t k = k0 + m;
            int a = s->ldir[k];
            dirs[m] = a;
            int64_t xf = (int64_t)wrap(by - EY[a], ny) * nx + wrap(bx - EX[a], nx);
            int64_t xff = (int64_t)wrap(by - 2 * EY[a], ny) * nx + wrap(bx - 2 * EX[a], nx);
            int f_ok = !s->solid[xf], ff_ok = f_ok && !s->solid[xff];
            double *v = in[m];
            v[0] = s->fs[a * N + b];
            v[1] = s->fs[OPP[a] * N + b];
            v[2] = f_ok ? s->fs[a * N + xf] : 0.0;
            v[3] = f_ok ? s->fs[OPP[a] * N + xf] : 0.0;
            v[4] = ff_ok ? s->fs[a * N + xff] : 0.0;
            v[5] = s->f[a * N + b];
            v[6] = s->rho[b];
            v[7] = s->ux[b];
            v[8] = s->uy[b];
            v[9] = f_ok ? s->ux[xf] : 0.0;
            v[10] = f_ok ? s->uy[xf] : 0.0;
            v[11] = s->luwx[k];
            v[12] = s->luwy[k];
            v[13] = f_ok ? 1.0 : 0.0;
            v[14] = ff_ok ? 1.0 : 0.0;
            double q = s->lq[k];
            if (s->rule == ORA_RULE_MLS && q < 0.5 && !f_ok) s->counters[0]++;
            if (s->rule == ORA_RULE_IBB_LINEAR && q < 0.5 && !f_ok) s->counters[1]++;
            if (s->rule == ORA_RULE_IBB_QUADRATIC &&
                ((q < 0.5 && !ff_ok) || (q >= 0.5 && !f_ok)))
                s->counters[2]++;
            inc[m] = ora_rule_incoming(s->rule, a, q, s->tau, v, s->rho[b],
                                       &chi[m], &br[m]);
            wall[m] = 2.0 * WT[a] * s->rho[b] * INV_CS2 *
                      (EX[a] * v[11] + EY[a] * v[12]);
        }
        if (s->fix == ORA_FIX_B || s->fix == ORA_FIX_BAO) {
            /* Scheme B, Eq. (22) (chi inside both sums); Bao et al.,
             * Eq. (23) (chi taken out).  A moving wall's momentum term is
             * not part of the balance (the paper's walls are at rest). */
            double num = 0.0, den = 0.0, mag = 0.0;
            for (int m = 0; m < n; ++m) {
                if (s->fix == ORA_FIX_B) {
                    num += chi[m] * in[m][0];
                    den += chi[m] * br[m];
                    mag += fabs(chi[m] * br[m]);
                } else {
                    num += in[m][0];
                    den += br[m];
                    mag += fabs(br[m]);
                }
            }
            if (den != 0.0 && fabs(den) > 1e-12 * mag) {
                double rho_s = num / den;
                for (int m = 0; m < n; ++m) {
                    int a = dirs[m];
                    inc[m] = ora_rule_incoming(s->rule, a, s->lq[k0 + m],
                                               s->tau, in[m], rho_s, NULL, NULL);
                }
            } else if (mag > 0.0) {
                s->counters[3]++; /* sums cancel: keep rho_b (no chi = 0
                                   * node is counted; it has no leak) */
            }
        }
        /* Eq. (15); a moving wall's momentum term (which the paper's
         * resting walls do not have) is added back so that only the rule's
         * own leak is measured and corrected. */
        double out_sum = 0.0, in_sum = 0.0;
        for (int m = 0; m < n; ++m) {
            out_sum += in[m][0];
            in_sum += inc[m] + wall[m];
            s->fn[OPP[dirs[m]] * N + b] = inc[m];
            /* momentum handed to the wall by this link */
            s->force[0] += EX[dirs[m]] * (in[m][0] + inc[m]);
            s->force[1] += EY[dirs[m]] * (in[m][0] + inc[m]);
        }
        double f0_before = s->fn[b];
        if (s->fix == ORA_FIX_A) {
            /* Eq. (18): the leak of Eq. (15) goes into the rest population */
            s->fn[b] = s->fn[b] + (out_sum - in_sum);
            if (s->fn[b] < 0.0) s->counters[4]++;
        }
        s->leaks[bi] = (out_sum - in_sum) - (s->fn[b] - f0_before);
    }
    /* 9. total mass */
    double m = 0.0, c = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (s->solid[i]) continue;
        for (int a = 0; a < 9; ++a) m = neumaier_add(m, s->fn[a * N + i], &c);
    }
    double *tmp = s->f;
    s->f = s->fn;
    s->fn = tmp;
    s->t++;
    *mass_out = m + c;
    return isfinite(m + c) ? 0 : -5;
}

int ora_step(ora_sim *s, int64_t n, double *mass_hist) {
    if (!s || n < 0) return -1;
    for (int64_t k = 0; k < n; ++k) {
        double m;
        int rc = one_step(s, &m);
        if (mass_hist) mass_hist[k] = m;
        if (rc) return rc;
    }
    return 0;
}

int ora_moments(ora_sim *s, double *rho, double *ux, double *uy) {
    if (!s) return -1;
    macroscopic(s);
    for (int64_t i = 0; i < s->N; ++i) {
        if (rho) rho[i] = s->solid[i] ? 0.0 : s->rho[i];
        if (ux) ux[i] = s->solid[i] ? 0.0 : s->ux[i];
        if (uy) uy[i] = s->solid[i] ? 0.0 : s->uy[i];
    }
    return 0;
}

double ora_total_mass(const ora_sim *s) {
    double m = 0.0, c = 0.0;
    for (int64_t i = 0; i < s->N; ++i) {
        if (s->solid[i]) continue;
        for (int a = 0; a < 9; ++a) m = neumaier_add(m, s->f[a * s->N + i], &c);
    }
    return m + c;
}

int64_t ora_time(const ora_sim *s) { return s->t; }

void ora_get_f(const ora_sim *s, double *f) {
    memcpy(f, s->f, (size_t)(9 * s->N) * sizeof(double));
}

void ora_set_f(ora_sim *s, const double *f) {
    memcpy(s->f, f, (size_t)(9 * s->N) * sizeof(double));
}

int64_t ora_last_leaks(const ora_sim *s, double *out, int64_t cap) {
    int64_t n = s->nb < cap ? s->nb : cap;
    for (int64_t i = 0; i < n; ++i) out[i] = s->leaks[i];
    return s->nb;
}

void ora_wall_force(const ora_sim *s, double out[2]) {
    out[0] = s->force[0];
    out[1] = s->force[1];
}

void ora_counters(const ora_sim *s, int64_t out[5]) {
    for (int i = 0; i < 5; ++i) out[i] = s->counters[i];
}
