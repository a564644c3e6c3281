/*
 * Plain FP64 CPU oracle for the two-phase D2Q9 lattice-Boltzmann step with
 * curved-wall rules and the mass-conservative corrections of Yu, Li & Wen,
 * "Modified curved boundary scheme for two-phase lattice Boltzmann
 * simulations" (arXiv:1908.09235).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a slow, obviously correct restatement of the paper.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU path.
 *
 * Every call returns 0 on success or a negative status:
 *   -1 invalid input, -4 singular parameter (Filippova-Haenel pole, Eq. 9),
 *   -5 non-finite total mass after a step.
 *
 * Directions (D2Q9): 0 rest; 1 (+1,0); 2 (0,+1); 3 (-1,0); 4 (0,-1);
 * 5 (+1,+1); 6 (-1,+1); 7 (-1,-1); 8 (+1,-1).  Node index = y*nx + x.
 * The domain is periodic in y, and in x unless open_x is set (flow past a
 * cylinder, Sec. 4.2: a uniform velocity inlet at x = 0 by the scheme of
 * Zou and He (1997) and a fully developed outlet at x = nx - 1); walls are
 * solid nodes.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_RULE_HALFWAY = 0, ORA_RULE_FH = 1, ORA_RULE_MLS = 2,
       ORA_RULE_IBB_LINEAR = 3, ORA_RULE_IBB_QUADRATIC = 4,
       ORA_RULE_ZHAO_YONG = 5 };
enum { ORA_FIX_NONE = 0, ORA_FIX_A = 1, ORA_FIX_B = 2, ORA_FIX_BAO = 3 };
enum { ORA_EOS_NONE = 0, ORA_EOS_EXP = 1, ORA_EOS_CS = 2 };
enum { ORA_COLL_BGK = 0, ORA_COLL_MRT = 1 };

typedef struct {
    int32_t nx, ny;
    const uint8_t *solid;          /* nx*ny, nonzero = solid                 */
    int64_t nlinks;                /* cut links, each (x,y) fluid, +e solid  */
    const int32_t *link_x, *link_y, *link_dir;
    const double *link_q;          /* wall fraction, Eq. 6, in (0,1]         */
    const double *link_uwx, *link_uwy; /* wall velocity at x_w (nullable)   */
    const double *rho_wall;        /* virtual wall density per node, read at
                                      solid nodes only (Sec. 3.2)          */
    int32_t eos;                   /* ORA_EOS_*                              */
    double eos_p[4];               /* EXP: psi0, rho0.  CS: a, b, R, T       */
    double G;                      /* interaction strength, Eq. 16           */
    double gx, gy;                 /* body acceleration, force = rho*g       */
    int32_t collision;             /* ORA_COLL_*                             */
    double tau;                    /* BGK relaxation time; MRT: 1/s_nu       */
    double mrt_s[9];               /* MRT rates in moment order              */
    int32_t rule, fix;
    const double *rho0;            /* initial density per node               */
    const double *ux0, *uy0;       /* initial velocity (nullable = 0)        */
    int32_t open_x;                /* 1: inlet at x = 0, outlet at nx - 1   */
    double inlet_u;                /* inlet velocity (x component; y = 0)    */
} ora_desc;

typedef struct ora_sim ora_sim;

int  ora_create(const ora_desc *d, ora_sim **out);
void ora_destroy(ora_sim *s);
/* n steps; mass_hist (nullable) receives M(t+1)..M(t+n). */
int  ora_step(ora_sim *s, int64_t n, double *mass_hist);
/* Moments of the current pre-collision state (Eq. 5); solid nodes get 0. */
int  ora_moments(ora_sim *s, double *rho, double *ux, double *uy);
double ora_total_mass(const ora_sim *s);
int64_t ora_time(const ora_sim *s);
/* f as [9][ny][nx] pre-collision populations. */
void ora_get_f(const ora_sim *s, double *f);
void ora_set_f(ora_sim *s, const double *f);
/* Per-boundary-node mass leak of the last step (Eq. 15) after the fix,
 * in the order of ascending node index; returns the number of nodes. */
int64_t ora_last_leaks(const ora_sim *s, double *out, int64_t cap);
/* Force exerted on the walls during the last step by momentum exchange
 * over the cut links: sum of e_a (f*_a(x_b, t) + f_abar(x_b, t+1)). */
void ora_wall_force(const ora_sim *s, double out[2]);
/* counters: [0] MLS u_f fallbacks, [1] IBB-L branch fallbacks,
 * [2] IBB-Q -> IBB-L fallbacks, [3] scheme-B degenerate nodes,
 * [4] scheme-A nodes with negative rest population. */
void ora_counters(const ora_sim *s, int64_t out[5]);

/* ---- pure functions exposed for the unit pins ---- */
void   ora_feq(double rho, double ux, double uy, double out[9]);
void   ora_guo(double tau, double ux, double uy, double Fx, double Fy,
               double out[9]);
void   ora_mrt_matrix(double M[81], double Minv[81]);
void   ora_collide(int32_t collision, double tau, const double s[9],
                   const double f[9], double rho, double ux, double uy,
                   double Fx, double Fy, double out[9]);
double ora_psi(int32_t eos, const double p[4], double G, double rho);
double ora_pressure_eos(int32_t eos, const double p[4], double rho);

/* Incoming population f_abar(x_b, t+1) of one cut link (Eqs. 7-14).
 * in[]: 0 f*_a(x_b)  1 f*_abar(x_b)  2 f*_a(x_f)  3 f*_abar(x_f)
 *       4 f*_a(x_ff)  5 f_a(x_b) pre-collision  6 rho_b  7 ubx  8 uby
 *       9 ufx 10 ufy 11 uwx 12 uwy  13 x_f fluid (0/1)  14 x_ff fluid
 * rho_eq: density in the fictitious equilibrium (rho_b, or rho_s of
 * scheme B / Bao).  chi_out, den_out (nullable): chi and the bracket
 * omega_a[...] of Eq. 22 for this link. */
double ora_rule_incoming(int32_t rule, int32_t dir, double q, double tau,
                         const double in[15], double rho_eq,
                         double *chi_out, double *bracket_out);

#ifdef __cplusplus
}
#endif
#endif
