/*
 * lbm2p: two-phase D2Q9 lattice-Boltzmann time step with curved walls and
 * mass-conservative boundary corrections, on AMD Instinct MI355X (gfx950).
 *
 * Method: Yu, Li & Wen, "Modified curved boundary scheme for two-phase
 * lattice Boltzmann simulations" (arXiv:1908.09235).  One time step is
 *   - the pseudopotential psi(rho) from an equation of state and the
 *     interaction force of Eq. (16), plus an optional body force rho*g;
 *   - collision, Eq. (2), with the equilibrium of Eq. (4) and the forcing
 *     term of Guo et al. that Sec. 3.2 cites (BGK, or a D2Q9
 *     multiple-relaxation-time form of the same step);
 *   - streaming, Eq. (3);
 *   - on every cut link, one curved-wall rule of Sec. 2.2: halfway
 *     bounce-back, Filippova-Haenel (Eqs. 7-10), Mei-Luo-Shyy (Eqs. 7, 8,
 *     10, 11), linear or quadratic Bouzidi (Eqs. 12, 13) or Zhao-Yong
 *     (Eq. 14);
 *   - at every boundary node, the leak of Eq. (15) and the correction of
 *     scheme A (Eq. 18), scheme B (Eqs. 20-22) or Bao et al. (Eq. 23).
 *
 * Conventions
 *   Lattice: D2Q9, directions 0 rest, 1 (+1,0), 2 (0,+1), 3 (-1,0),
 *   4 (0,-1), 5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1).
 *   Host arrays of nodes are row-major with index y*nx + x.
 *   The domain is periodic in y, and in x unless open_x is set (Sec. 4.2:
 *   a uniform velocity inlet at x = 0 by the scheme of Zou and He (1997),
 *   a fully developed outlet at x = nx - 1); walls are solid nodes.  A cut link
 *   (x, y, dir) joins a fluid node to a solid node at (x, y) + e_dir; every
 *   such adjacency must be listed exactly once.
 *
 * Ownership: the caller owns every array it passes; lbm_create_domain
 *   copies what it needs and keeps no pointer.  The domain owns all device
 *   memory until lbm_destroy.  Output arrays are caller-allocated.
 *
 * Errors: every call returns an lbm_status; nothing throws or aborts.  On
 *   error the outputs are untouched and nothing is leaked.
 *
 * Threading: one host thread per domain at a time.  Several domains may
 *   share a device and a stream.
 */
#ifndef LBM2P_H
#define LBM2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument or inconsistent geometry       */
    LBM_ENOMEM = -2,     /* device or host allocation failed                 */
    LBM_EDEVICE = -3,    /* a HIP runtime call failed                        */
    LBM_ESINGULAR = -4,  /* Filippova-Haenel with q < 1/2 at tau = 1 (Eq. 9) */
    LBM_EUNSTABLE = -5   /* a step produced a non-finite total mass          */
} lbm_status;

enum lbm_rule {
    LBM_RULE_HALFWAY = 0,        /* f_abar(x_b,t+1) = f*_a(x_b,t)            */
    LBM_RULE_FH = 1,             /* Eqs. 7-10                                */
    LBM_RULE_MLS = 2,            /* Eqs. 7, 8, 10, 11                        */
    LBM_RULE_IBB_LINEAR = 3,     /* Eq. 12                                   */
    LBM_RULE_IBB_QUADRATIC = 4,  /* Eq. 13                                   */
    LBM_RULE_ZHAO_YONG = 5       /* Eq. 14                                   */
};

enum lbm_fix {
    LBM_FIX_NONE = 0,
    LBM_FIX_A = 1,    /* Eq. 18: leak added to the rest population          */
    LBM_FIX_B = 2,    /* Eqs. 20-22: fictitious density balancing the node  */
    LBM_FIX_BAO = 3   /* Eq. 23: Bao et al.'s density (chi outside the sum) */
};

enum lbm_eos {
    LBM_EOS_NONE = 0, /* single phase: no interaction force                */
    LBM_EOS_EXP = 1,  /* psi = p0 exp(-p1/rho)                              */
    LBM_EOS_CS = 2    /* Carnahan-Starling, p = (a, b, R, T):
                         psi = sqrt(2 (p_CS(rho) - rho/3) / G)              */
};

enum lbm_collision { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };

/* Precision forms.  The paper fixes none (its runs are double precision);
 * every form computes the same step.  The boundary rules, boundary sums and
 * total mass stay FP64 in every form.  The deviation forms store
 * g_a = f_a - w_a rho_ref (w_a the lattice weights of Eq. 4) so that the
 * stored number carries only the departure from a uniform fluid at rest. */
enum lbm_storage {
    LBM_STORE_F64 = 0,         /* FP64 populations, FP64 arithmetic        */
    LBM_STORE_F32 = 1,         /* FP32 populations, FP64 arithmetic        */
    LBM_STORE_F32_ARITH32 = 2, /* FP32 populations, FP32 arithmetic        */
    LBM_STORE_F32DEV = 3,      /* FP32 deviations, FP32 arithmetic         */
    LBM_STORE_F16DEV = 4,      /* FP16 (IEEE binary16) deviations, FP32
                                  arithmetic                              */
    LBM_STORE_F16NODE = 5      /* FP16 deviations g_a = f_a - w_a r(x) from a
                                  per-node reference r: the current density
                                  of the node x whose slot holds g (an FP32
                                  plane after the nine population planes,
                                  rewritten by every update; a solid node
                                  that receives incoming populations takes
                                  the density of one fluid node next to it;
                                  initially rho0).  One FP32 read and one
                                  write of r per update on top of the FP16
                                  traffic; FP32 arithmetic; rho_ref is
                                  ignored                                 */
};

/* One cut link (40 bytes). */
typedef struct {
    int32_t x, y;       /* fluid boundary node x_b                          */
    int32_t dir;        /* 1..8; x_b + e_dir is solid                       */
    int32_t reserved;   /* must be 0                                        */
    double q;           /* wall fraction of Eq. 6, 0 < q <= 1               */
    double uw[2];       /* wall velocity at the cut point (0 for the paper's
                           resting walls); only HALFWAY, FH, MLS accept it  */
} lbm_link;

typedef struct {
    int32_t nx, ny;            /* lattice size, each >= 3, nx*ny < 2^30;
                                  one state buffer must stay below
                                  2^32 - 256 bytes: nine planes of
                                  pitch*ny + 256 elements (pitch = nx
                                  rounded up to 64), plus an FP32 plane of
                                  that size for the FP16 per-node form
                                  (about 59 M nodes in FP64, 119 M in
                                  FP32, 195 M FP16 per-node)            */
    const uint8_t *solid;      /* host, nx*ny, nonzero = solid node         */
    const lbm_link *links;     /* host, nlinks cut links                    */
    int64_t nlinks;
    const double *rho_wall;    /* host, nx*ny virtual wall density read at
                                  solid nodes (contact angle, Sec. 3.2);
                                  NULL: rho_wall_const everywhere          */
    double rho_wall_const;
    int32_t eos;               /* enum lbm_eos                              */
    int32_t collision;         /* enum lbm_collision                        */
    double eos_param[4];       /* EXP: psi0, rho0.  CS: a, b, R, T          */
    double G;                  /* interaction strength of Eq. 16 (< 0 is
                                  attractive); ignored for EOS_NONE         */
    double gravity[2];         /* body force per unit density               */
    double tau;                /* relaxation time (> 1/2); for MRT the
                                  shear rates mrt_s[7], mrt_s[8] must equal
                                  1/tau                                     */
    double mrt_s[9];           /* MRT rates, moments (rho, e, eps, jx, qx,
                                  jy, qy, pxx, pxy) of Lallemand & Luo      */
    int32_t rule;              /* enum lbm_rule                             */
    int32_t fix;               /* enum lbm_fix; B and BAO need FH or MLS    */
    int32_t storage;           /* enum lbm_storage                          */
    int32_t open_x;            /* 0 periodic in x; 1 velocity inlet at x = 0
                                  and outlet at x = nx - 1 (single phase
                                  only; nx >= 8; columns 0..2 and
                                  nx-3..nx-1 fluid)                        */
    const double *rho0;        /* host, nx*ny initial density (> 0 on fluid)*/
    const double *ux0, *uy0;   /* host, nx*ny initial velocity, or NULL     */
    int64_t history_capacity;  /* mass-history ring entries; 0 = 1048576   */
    void *stream;              /* hipStream_t for all work, NULL = default  */
    int32_t tile_w;            /* launch shape of the main kernel: columns
                                  per workgroup (64, 128 or 256; 0 = auto)  */
    int32_t tile_h;            /* rows per workgroup (0 = auto)             */
    double rho_ref;            /* reference density of the deviation forms
                                  (>= 0; 0 = mean of rho0 over fluid nodes);
                                  ignored by the other forms              */
    double inlet_u;            /* open_x: inlet velocity, x component
                                  (|inlet_u| < 1; the y component is 0)    */
} lbm_desc;

typedef struct lbm_domain lbm_domain;

/* Validate the descriptor, build the boundary tables, upload the state and
 * compute f*(0) from f(0) = f_eq(rho0, u0).  Errors: LBM_EINVAL (sizes,
 * tau <= 1/2, a bad or missing or duplicate link, q outside (0,1], a
 * moving wall with a rule that does not support it, rho0 <= 0 on a fluid
 * node, psi^2 < 0 at rho0 or at a wall density, FIX_B/BAO with a rule
 * other than FH/MLS, MRT shear rates != 1/tau), LBM_ESINGULAR, LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_create_domain(const lbm_desc *desc, lbm_domain **out);

/* Advance n >= 0 steps and wait for them.  One step is the whole method
 * of Secs. 2-4: psi and the interaction force (Eq. 16, Sec. 3.2) with the
 * body force, the moments (Eq. 5), the collision with the Guo forcing term
 * (Eqs. 1-2, 4; MRT as in Sec. 3.2), the pull streaming (Eq. 3), the rule
 * of every cut link (Eqs. 6-14), the correction at every boundary node
 * (Eqs. 15, 17-23) and the total mass.  Steps are enqueued on the domain's
 * stream (as HIP graph replays once the step count repeats) and no host
 * data moves.  n = 0 does nothing.  LBM_EUNSTABLE names the first step
 * whose total mass was not finite (see lbm_unstable_step); further steps
 * still run on the non-finite state and report the same first step. */
int lbm_step(lbm_domain *d, int64_t n);

/* As lbm_step, without waiting; lbm_sync waits and reports the status. */
int lbm_step_async(lbm_domain *d, int64_t n);
int lbm_sync(lbm_domain *d);

/* Density and velocity of Eq. 5 at the current time into host arrays of
 * nx*ny doubles (any may be NULL); solid nodes get 0. */
int lbm_moments(lbm_domain *d, double *rho, double *ux, double *uy);

/* As lbm_moments into device arrays of nx*ny doubles, on the domain's
 * stream, without waiting. */
int lbm_moments_device(lbm_domain *d, double *rho, double *ux, double *uy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): as
 * lbm_moments_device, but staged through a buffer the library holds on
 * every GPU it runs on from load time to process exit (3 x 2^21 doubles,
 * 48 MiB), so the call allocates nothing, with or without an earlier
 * lbm_moments call.  Domains of more than 2^21 nodes (nx*ny) get
 * LBM_EINVAL.  Every call on one GPU shares that buffer: calls that
 * overlap on one GPU (different streams, different host threads) race and
 * must be serialised by the caller; calls on one stream are ordered.  The
 * copies into rho, ux, uy are enqueued on the domain's stream. */
int lbm_moments_device_noalloc(lbm_domain *d, double *rho, double *ux, double *uy);

/* Total mass M(t) = sum over fluid nodes of sum_a f*_a (FP64, summed in a
 * fixed order, so equal states give equal bits): the m of Sec. 3.2, whose
 * ratio m/m0 the paper plots in Figs. 4-8.  The post-collision
 * populations carry the same mass as the pre-collision ones. */
int lbm_total_mass(lbm_domain *d, double *out);

/* Current time step count. */
int lbm_time(lbm_domain *d, int64_t *t);

/* The last min(t+1, capacity, cap) total masses M(t) (as lbm_total_mass;
 * the m(t) whose ratio to m(0) Sec. 3.2 and Figs. 4-8 follow) in time
 * order into out[0 .. *n_written - 1], oldest first; the ring holds the
 * capacity given at creation.  cap < 0, or a NULL out or n_written, gives
 * LBM_EINVAL. */
int lbm_mass_history(lbm_domain *d, double *out, int64_t cap,
                     int64_t *n_written);

/* Step index of the first non-finite total mass, or -1. */
int lbm_unstable_step(lbm_domain *d, int64_t *step);

/* Checkpoint: with buf == NULL, *bytes receives the size; otherwise the
 * state is written if *bytes is large enough (else LBM_EINVAL).  Restoring
 * it into a domain built from the same descriptor resumes bit-exactly. */
int lbm_get_state(lbm_domain *d, void *buf, size_t *bytes);
int lbm_set_state(lbm_domain *d, const void *buf, size_t bytes);

/* Per-kernel timing: with every > 0, the boundary and main launches of
 * every every-th step record their own start and end on HIP events of the
 * domain's stream (the dispatch's timestamps, as a kernel profiler reads
 * them; no host synchronisation until 1024 samples are pending);
 * lbm_kernel_times returns the summed durations (ms) and sample counts
 * since profiling was last set.  every = 0 switches it off. */
int lbm_set_profiling(lbm_domain *d, int every);
int lbm_kernel_times(lbm_domain *d, double *main_ms, int64_t *main_count,
                     double *boundary_ms, int64_t *boundary_count);

/* Force exerted on the walls during the last step, by momentum exchange
 * over the cut links (Sec. 4.2): out = sum of e_a (f*_a(x_b, t) +
 * f_abar(x_b, t + 1)), summed in a fixed order.  Zero before the first
 * step. */
int lbm_wall_force(lbm_domain *d, double out[2]);

/* Scheme A (Eq. 18) adds a node's leak to its rest population, which can
 * then turn negative; nothing clamps it.  *count receives the number of
 * (boundary node, step) pairs where it did, since creation or the last
 * lbm_set_state (0 under the other fixes).  Waits for the domain's
 * stream. */
int lbm_negative_rest(lbm_domain *d, int64_t *count);

/* Steps per pass of the main kernel.  With 2, one launch advances two time
 * steps: the intermediate populations stay in on-chip memory and the wall
 * rules and corrections of the second step (Eqs. 7-15, 18, 20-23) are
 * evaluated inside the launch, so the populations cross HBM once per two
 * updates; the results are bit-identical to single steps.  Available for
 * the FP32 and FP16-deviation storage forms (not the FP16 per-node one),
 * periodic domains, every rule but Zhao-Yong and the quadratic
 * interpolation, and link tables of fewer than 2^23 - 1 slots (LBM_EINVAL
 * otherwise);
 * the default is 1.  tile_h is the two-step kernel's rows per workgroup
 * (0 = default 16, at least 4).  An odd step count ends with a
 * single step.  After a two-step pass the moments and the wall force of
 * the last step come from a replay of the intermediate step, in buffers
 * held since creation. */
int lbm_set_steps_per_pass(lbm_domain *d, int32_t steps, int32_t tile_h);

/* Autotuner for lbm_set_steps_per_pass: runs steps_per_trial >= 2 steps
 * untimed (they capture the step graphs), then steps_per_trial steps timed
 * on the domain's stream, under each setting -- one step per pass, and
 * where two are available two per pass with tiles of 4, 6, 8, 12, 16 and
 * 24 rows -- keeps the fastest and reports in out: steps per pass, rows
 * per tile (of the single-step kernel when one step per pass wins),
 * microseconds per step.  The steps count as steps of the domain (2 x
 * steps_per_trial per setting); every setting gives the same results bit
 * for bit.  Waits for the domain's stream.  LBM_EINVAL for NULL arguments
 * or steps_per_trial < 2; LBM_EUNSTABLE (out filled) if a step was
 * unstable; on a device error the caller's setting is restored. */
int lbm_tune_steps_per_pass(lbm_domain *d, int64_t steps_per_trial, int32_t out[3]);
int lbm_get_steps_per_pass(lbm_domain *d, int32_t *steps, int32_t *tile_h);

/* Scheme B (Eq. 22) and Bao et al. (Eq. 23) divide by a sum over the
 * node's links that can cancel when tau >= 2 (chi < 0 for q < 1/2); where
 * it vanishes or falls below 1e-12 of the sum of its terms' magnitudes the
 * node keeps rho_b for that step (a node whose every chi is 0 has no leak
 * and is not counted).  *count receives the number of such (boundary
 * node, step) pairs since creation or the last lbm_set_state.  Waits for
 * the domain's stream. */
int lbm_degenerate_b(lbm_domain *d, int64_t *count);

/* Facts about the built domain: [0] fluid nodes, [1] cut links,
 * [2] boundary nodes, [3] bytes of device memory held, [4] tile_w,
 * [5] tile_h, [6] main-kernel workgroups, [7] boundary-rule fallbacks
 * (x_f or x_ff solid) taken per step. */
int lbm_info(lbm_domain *d, int64_t out[8]);

void lbm_destroy(lbm_domain *d);
const char *lbm_status_string(int status);

/* ------------------------------------------------------------------------
 * Batched form: many independent domains (instances) advanced together.
 * Each instance is a complete domain as above (its own geometry, EOS
 * parameters, tau or MRT rates, rule, fix and state) and computes exactly
 * what lbm_step computes for it alone.  All instances of a batch share the
 * storage form and the EOS kind.  Device memory for all of them comes from
 * one arena allocated at creation; instances are built on a stream of the
 * batch's own while earlier work runs on the compute stream.  A step of the
 * batch is three launches over all instances (boundary pass, main pass,
 * per-instance mass reduction), replayed from a captured HIP graph.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

typedef struct {
    int32_t storage;        /* enum lbm_storage of every instance          */
    int32_t eos;            /* enum lbm_eos of every instance              */
    int32_t max_instances;  /* instance slots, 1 .. 2^20                    */
    int32_t tile_w;         /* main-pass tile columns: 64, 128, 256 (0=256) */
    int32_t tile_h;         /* main-pass tile rows: >= 8 (0 = 16)           */
    int32_t persistent;     /* 1: a resident grid takes tiles from per-XCD
                               queues; 0: one workgroup per tile           */
    int32_t graph_steps;    /* steps per captured graph (0 = 32; < 0: no
                               graph, plain launches)                      */
    int32_t ring;           /* rows of population loads per lane of the
                               main pass, the row computed and those in
                               flight: 2, 3 or 4 (0 = 3; the FP16 per-node
                               form accepts 0 or 3 only)                   */
    int64_t arena_bytes;    /* device memory for all instances (> 0)        */
    void *stream;           /* compute stream (NULL: the batch makes one)   */
} lbm_batch_desc;

/* Errors: LBM_EINVAL (a field out of range), LBM_ENOMEM (the arena or the
 * tables), LBM_EDEVICE. */
int lbm_batch_create(const lbm_batch_desc *bd, lbm_batch **out);

/* Build an instance from a descriptor (as lbm_create_domain: same
 * validation and errors, and open_x must be 0; desc->stream, tile_w and
 * tile_h are ignored) that
 * will run `steps` steps and then stop.  *slot receives its slot index.
 * LBM_ENOMEM when no slot is free or the arena has no room for it; the
 * batch is unchanged then.  The instance joins the next lbm_batch_run. */
int lbm_batch_add(lbm_batch *b, const lbm_desc *desc, int64_t steps, int32_t *slot);

/* Enqueue n steps for every instance (each stops after its own count) on
 * the compute stream; waits for the previous run first. */
int lbm_batch_run(lbm_batch *b, int64_t n);
int lbm_batch_sync(lbm_batch *b);

/* Per instance, after waiting for the batch: the current step, the steps
 * still to run, and the first step with a non-finite total mass (or -1;
 * an unstable instance stops). */
int lbm_batch_status(lbm_batch *b, int32_t slot, int64_t *t, int64_t *remaining,
                     int64_t *unstable_step);
/* As lbm_moments and lbm_mass_history, for one instance. */
int lbm_batch_moments(lbm_batch *b, int32_t slot, double *rho, double *ux, double *uy);
int lbm_batch_mass_history(lbm_batch *b, int32_t slot, double *out, int64_t cap,
                           int64_t *n_written);
/* Free an instance's memory and its slot. */
int lbm_batch_remove(lbm_batch *b, int32_t slot);

/* Autotuner: runs steps_per_trial real steps of the batch (after one
 * warm-up step) under each main-pass configuration -- columns per
 * workgroup (tile_w 64/128/256), rows per lane (tile_h 8/16/32),
 * persistent or not, and rows of population loads each lane keeps in
 * flight ahead of the row it computes (1, 2 or 3: a ring of 2, 3 or 4
 * rows of nine populations; the FP16 per-node form always 2) -- keeps the
 * fastest and reports it in out: tile_w, tile_h, persistent, microseconds
 * per step, ring rows.  The steps count as steps of the instances; results
 * do not depend on the configuration.  A batch with no instances keeps its
 * configuration and reports 0 microseconds. */
int lbm_batch_tune(lbm_batch *b, int64_t steps_per_trial, int32_t out[5]);

/* [0] instances, [1] main-pass tiles, [2] link blocks, [3] arena bytes,
 * [4] arena bytes in use, [5] tile_w, [6] tile_h, [7] persistent. */
int lbm_batch_info(lbm_batch *b, int64_t out[8]);
void lbm_batch_destroy(lbm_batch *b);

/* ------------------------------------------------------------------------
 * Served form: a request queue in front of a batch (continuous batching).
 * lbm_server_submit queues a request (a descriptor and a step count); the
 * arrays the descriptor points to must stay valid until the request is
 * admitted.  Each lbm_server_progress call is one scheduling round: it
 * waits for the chunk of steps in flight, reports the requests that
 * finished, launches the next chunk_steps steps for every resident request,
 * and while that chunk runs admits queued requests in arrival order as long
 * as their instance fits in the arena and a slot is free.  A finished
 * request keeps its memory until lbm_server_release.
 * ------------------------------------------------------------------------ */
typedef struct lbm_server lbm_server;

int lbm_server_create(const lbm_batch_desc *bd, int64_t chunk_steps, lbm_server **out);
int lbm_server_submit(lbm_server *s, const lbm_desc *desc, int64_t steps, int64_t *id);
/* done_ids receives the ids of finished requests not reported before, at
 * most cap of them (*n_done); any others are reported by later calls. */
int lbm_server_progress(lbm_server *s, int64_t *done_ids, int64_t cap, int64_t *n_done);
/* A finished request: its final rho, u (host arrays of nx*ny, any may be
 * NULL), mass[0] = M(0) (NaN if it left the history ring) and mass[1] =
 * the final M, the steps it ran and its first unstable step (or -1). */
int lbm_server_result(lbm_server *s, int64_t id, double *rho, double *ux, double *uy,
                      double mass[2], int64_t *steps_done, int64_t *unstable_step);
int lbm_server_release(lbm_server *s, int64_t id);
/* [0] queued, [1] running, [2] finished and not released, [3] arena bytes
 * in use, [4] arena bytes, [5] chunks launched, [6] admitted, [7] rejected
 * (invalid descriptors, or too large for the arena). */
int lbm_server_info(lbm_server *s, int64_t out[8]);
void lbm_server_destroy(lbm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* LBM2P_H */
