/*
 * pd.h -- C ABI of libpd: the PeriDEM step loop on an AMD MI355X (gfx950).
 *
 * The library advances a 2-D aggregate of deformable particles by the
 * method of Bhattacharya & Lipton, "Simulating grain shape effects and
 * damage in granular media using PeriDEM":
 *   - intra-particle bond-based peridynamic force with irreversible bond
 *     breaking (Sec. 3, eq. peri, eq. pmb, Table tab:2d-peri, Sec. 3.1);
 *   - reference bonds restricted to segments that stay inside the particle,
 *     found once by the extended-boundary and cusp-bisector test of Sec. 5;
 *   - contact between nodes closer than R_c, evaluated every step from exact
 *     distances over per-node candidate lists (all pairs within R_c plus a
 *     skin), which a radix-sorted cell list rebuilds when a node has moved
 *     half the skin or a bond broke (Algorithm alg:buildtree, inter-particle
 *     neighbour sets); skin 0 runs the cell search every step.  Short-range
 *     repulsion (Sec. 4.1), regularized
 *     Coulomb friction (Sec. 4.2), normal damping (Sec. 4.3) and self-contact
 *     between unbonded nodes of one particle (Sec. 4.4);
 *   - analytic contact with the four walls of a rectangular container whose
 *     top wall may move down (Sec. 4.5, eq. wall-total);
 *   - velocity-Verlet integration (Sec. 6.1, Algorithm alg:buildtree);
 *   - optionally, a learned reduced-order closure of the bond force for
 *     particles of repeated shapes (pd_closure_*; not part of the paper).
 * The problem statement is the initial value problem eq. pdmotion with the
 * forces of eq. full.
 *
 * Conventions
 *   - SI units per unit thickness: nodal "volume" is an area (m^2), density
 *     kg/m^3, nodal force N/m (Sec. 7 intro: in 2-D volume means area).
 *   - Arrays are structure-of-arrays, one double per node unless stated.
 *   - Every call returns pd_status; no exception crosses the ABI.  After an
 *     error, pd_last_error() gives a message.  PD_E_NONFINITE and
 *     PD_E_ESCAPED are sticky until pd_set_state().
 *   - Ownership: the caller owns every input and may free it when pd_setup
 *     returns (the library deep-copies to device memory).  The context owns
 *     all device memory it allocates.  Output buffers are caller-allocated:
 *     host pointers, or device pointers when on_device = 1.
 *   - Concurrency: one context is used by one host thread at a time.  Work is
 *     issued on the stream given at setup.  With NULL the library runs on a
 *     stream of its own (graphs cannot be captured on the legacy default
 *     stream); a call that reads or writes caller device buffers first waits
 *     for the work already issued on the legacy default stream.  Calls return
 *     when their work is complete.
 *   - Determinism: sums run in a fixed order (gather only, no floating-point
 *     atomics), so the same inputs on the same device give bitwise equal
 *     results for a fixed tuning.
 */
#ifndef PD_H
#define PD_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pd_ctx pd_ctx;

typedef enum {
    PD_OK = 0,
    PD_E_INVALID = 1,   /* invalid argument or problem description */
    PD_E_NOMEM = 2,     /* device or host allocation failed */
    PD_E_DEVICE = 3,    /* HIP runtime error */
    PD_E_NONFINITE = 4, /* a displacement or velocity became NaN/Inf */
    PD_E_ESCAPED = 5,   /* a node went through a wall by R_c or more */
    PD_E_STATE = 6      /* call not valid in the current state */
} pd_status;

enum { PD_MICRO_CONST = 0, PD_MICRO_CONIC = 1 };           /* Table tab:2d-peri */
enum { PD_PREC_FP64 = 0, PD_PREC_FP32_FORCE = 1 };         /* force arithmetic */
enum { PD_KN_SELF_CONSISTENT = 0, PD_KN_PAPER_3D = 1 };    /* normal contact stiffness */

/* force terms of eq. full, for pd_forces */
enum {
    PD_TERM_PD = 1,    /* peridynamic bond force, eq. peri */
    PD_TERM_SELF = 2,  /* self-contact: repulsion, damping, friction (Sec. 4.4) */
    PD_TERM_NBR = 4,   /* other particles: repulsion, damping, friction */
    PD_TERM_WALL = 8,  /* container walls (Sec. 4.5) */
    PD_TERM_BODY = 16, /* body force rho g */
    PD_TERM_ALL = 31
};

typedef struct {
    double rho;     /* mass density, kg/m^3 */
    double bulk_k;  /* bulk modulus k, Pa */
    double young_E; /* Young's modulus; <= 0: E = 2 k (1 - nu) = 4k/3 (nu = 1/3 in 2-D) */
    double Gc;      /* critical energy release rate, J/m^2 */
    double horizon; /* peridynamic horizon eps, m */
    int32_t micro;  /* PD_MICRO_CONST (w = 1) or PD_MICRO_CONIC (w = 1 - |xi|/eps) */
} pd_material;

typedef struct {
    int32_t n_nodes, n_particles, n_aggregates, n_materials;
    const double *x, *y;                /* [n_nodes] reference coordinates */
    const double *vol;                  /* [n_nodes] nodal area */
    const int32_t *particle_offset;     /* [n_particles+1]; nodes of a particle are contiguous */
    const int32_t *particle_material;   /* [n_particles] index into materials */
    const int32_t *particle_aggregate;  /* [n_particles] or NULL (all 0); aggregates never interact */
    const pd_material *materials;       /* [n_materials] */
    const int32_t *loop_offset;         /* [n_particles+1] range of boundary loops per particle */
    const int32_t *loop_vertex_offset;  /* [n_loops+1] range of vertices per loop */
    const double *loop_xy;              /* interleaved vertices; outer loop counter-clockwise,
                                           holes clockwise; a particle with no loop is treated
                                           as convex (no bond is filtered) */
    const double *u0x, *u0y, *v0x, *v0y; /* [n_nodes] initial displacement/velocity or NULL (0) */
    double contact_radius;              /* R_c */
    double friction_mu;                 /* Coulomb coefficient mu */
    double damping_ratio;               /* r_d in [0, 1] */
    int32_t kn_mode;                    /* PD_KN_SELF_CONSISTENT: K_n = c_w / R_c;
                                           PD_KN_PAPER_3D: K_n = 18 k / (pi eps^5) */
    const double *box;                  /* [n_aggregates*4] xlo, xhi, ylo, yhi at t = 0 */
    const double *top_wall_speed;       /* [n_aggregates] downward speed of the top wall, or NULL */
    double gravity_x, gravity_y;        /* body acceleration g */
    double dt;                          /* time step */
    int32_t precision;                  /* PD_PREC_FP64 or PD_PREC_FP32_FORCE */
    void *hip_stream;                   /* hipStream_t for all work, or NULL */
} pd_problem;

/* Tuning of the launch configuration.  Results are bitwise identical for
 * every block size, staging and graph choice, and equal within rounding for
 * every cell factor, skin, lane count and wall pass (the contact set itself
 * never changes: it is evaluated from exact distances every step; the lane
 * count changes the order of the per-node sums, and so does the wall pass
 * for a node's wall regions at one or two lanes per node). */
typedef struct {
    int32_t block_nodes;  /* nodes per workgroup of the force kernel: 64, 128 or 256 */
    double cell_factor;   /* cell side / search radius, >= 1 */
    int32_t use_lds;      /* stage bond partners' coordinates in LDS (1) or read through cache (0) */
    int32_t use_graph;    /* replay steps as a captured HIP graph (1) or launch directly (0) */
    double skin_factor;   /* contact candidates within R_c (1 + skin_factor) are listed per node
                             and the list is rebuilt (cell-key radix sort) when a node has moved
                             half the skin or a bond broke; 0: search the cells every step */
    int32_t lanes_per_node; /* threads per node of the step kernel with candidate lists: 4 (short
                               chains of dependent work, small problems), 2 or 1 (per-node work
                               done once, large problems); other evaluations use 4 */
    int32_t wall_pass;    /* with candidate lists and the closure off: 1 evaluates the wall
                             forces (Sec. 4.5) of the nodes near a wall and the contact forces
                             (Sec. 4.1-4.4) of the nodes with candidates in a pass of their own
                             before each step kernel (one more launch per step, a step kernel
                             with fewer registers: large problems); 0 inside the step kernel */
} pd_tuning;

/* Builds the context: validates the problem, copies it to the device,
 * computes per-material constants (Table tab:2d-peri; K_n of Sec. 4.1),
 * builds the reference bonds (Algorithm alg:buildtree, reference neighbour
 * sets: same particle, |x' - x| < eps) minus the non-bonds of Sec. 5, and
 * evaluates the forces at t = 0 (applying the break rule) to obtain the
 * initial acceleration a0 = F / (rho V) + g.
 * Errors: PD_E_INVALID (empty particle, unordered offsets, dt <= 0,
 * R_c <= 0, bad material index, node outside its box by R_c or more),
 * PD_E_NOMEM, PD_E_DEVICE. */
pd_status pd_setup(const pd_problem *p, pd_ctx **out);

/* Releases all device memory of the context. NULL is allowed. */
void pd_destroy(pd_ctx *c);

/* Message of the last error on this context (never NULL). */
const char *pd_last_error(const pd_ctx *c);

/* n_steps iterations of Algorithm alg:buildtree: u += dt v + dt^2/2 a;
 * contact sets at the new positions; forces with the velocities of the
 * previous step; a = F / (rho V) + g; v += dt/2 (a_old + a).  Returns after
 * the work is complete.  Errors: PD_E_NONFINITE, PD_E_ESCAPED (sticky),
 * PD_E_DEVICE, PD_E_INVALID (n_steps < 0). */
pd_status pd_step(pd_ctx *c, int64_t n_steps);

/* Force density rho u'' by term (eq. full; nodal force divided by nodal
 * area) at the current state, summed over the terms in term_mask.  The
 * break rule is applied to the evaluation but not committed.  fx, fy:
 * [n_nodes], host or device (on_device = 1). */
pd_status pd_forces(pd_ctx *c, uint32_t term_mask, double *fx, double *fy, int32_t on_device);

/* pd_forces for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same evaluation and the same results as pd_forces(..., on_device = 1),
 * with the per-term workspace in a fixed array of 32 MiB that each device
 * the library runs on holds from its first pd_setup until the process ends
 * (10 doubles per node: at most 419 430 nodes).  The call allocates nothing.
 * fx, fy: [n_nodes] device buffers on the context's device.
 * Errors: PD_E_INVALID for a null output or a problem with more nodes than
 * the workspace holds (nothing is launched), PD_E_DEVICE.
 * Every call on one device shares that device's workspace, which keeps the
 * last call's contents (each call writes every entry it reads): calls that
 * overlap on one device, from contexts on different streams or threads,
 * race and must be serialised by the caller. */
pd_status pd_forces_noalloc(pd_ctx *c, uint32_t term_mask, double *fx, double *fy);

/* Damage of each node (Sec. 3.1): broken bonds / reference bonds, and the
 * number of broken directed bonds.  phi: [n_nodes] host or device, or NULL. */
pd_status pd_damage(pd_ctx *c, double *phi, int64_t *n_broken_directed, int32_t on_device);

/* Reference bonds as CSR (directed, columns ascending): row[n_nodes+1],
 * col[pd_n_bonds()], host memory. */
int64_t pd_n_bonds(const pd_ctx *c);
pd_status pd_bonds(pd_ctx *c, int32_t *row, int32_t *col);

/* Contact set at the current positions: unordered pairs (i < j) of nodes of
 * one aggregate with |p_i - p_j|^2 < R_c^2, sorted by i then j.  Writes at
 * most cap pairs to host arrays pi, pj; *count receives the set size. */
pd_status pd_contacts(pd_ctx *c, int32_t *pi, int32_t *pj, int64_t cap, int64_t *count);

/* State copy (host arrays of n_nodes; broken: one byte per directed bond in
 * CSR order; step: number of steps taken).  Any pointer may be NULL. */
pd_status pd_get_state(pd_ctx *c, double *ux, double *uy, double *vx, double *vy, double *ax,
                       double *ay, uint8_t *broken, int64_t *step);
pd_status pd_set_state(pd_ctx *c, const double *ux, const double *uy, const double *vx,
                       const double *vy, const double *ax, const double *ay,
                       const uint8_t *broken, int64_t step);

/* Counters accumulated since setup while counting is on (pd_set_counting):
 * [0] inter-particle pairs, [1] self-contact pairs, [2] sticking, [3] sliding,
 * [4] wall regions, [5] coincident pairs skipped, [6] bonds broken (directed),
 * [7] steps taken. */
pd_status pd_counters(pd_ctx *c, int64_t out[8]);
pd_status pd_set_counting(pd_ctx *c, int32_t on);

/* Launch configuration (see pd_tuning). */
pd_status pd_get_tuning(const pd_ctx *c, pd_tuning *t);
pd_status pd_set_tuning(pd_ctx *c, const pd_tuning *t);

/* Autotuner: for each candidate configuration, starting from a copy of the
 * state and bonds, two warm-up steps and then two windows of steps_per_trial
 * steps, the shorter window counting; the pass of walls and contact
 * candidates (wall_pass = 1) is tried on the three fastest list-mode
 * candidates, and the four fastest of all are timed again over windows of
 * 3 * steps_per_trial steps; the fastest of those is kept.  The state, bonds
 * and counters are restored afterwards.  chosen may be NULL. */
pd_status pd_autotune(pd_ctx *c, int32_t steps_per_trial, pd_tuning *chosen);

/* Kernel timing: runs n_steps steps and records HIP events on the
 * context's stream; ms[k] receives the mean duration per launch of kernel
 * class k and launches[k] the number of launches timed:
 *   0 cell keys (with one key per thread also the first radix pass's digit
 *   count), 1 radix histogram, 2 radix digit scan, 3 radix scatter,
 *   4 cell starts, 5 force + integrate (one per step), 6 candidate-list
 *   build, 7 the pass of walls and contact candidates before each step
 *   kernel (n_out >= 8; tuning wall_pass = 1 only).
 * Search kernels are bracketed one by one.  With candidate lists (skin > 0)
 * the force kernel is timed over runs of up to 64 steps issued as pd_step
 * issues them (one graph replay when the tuning's use_graph is set, else
 * back-to-back launches), events at the ends of each run: its mean is the
 * replay's time per step and excludes per-launch event overhead.  With the
 * wall pass the run's launches are issued one by one, each bracketed by
 * events, so that class 5 is the step kernel's own duration.
 * (n_out >= 7) */
pd_status pd_time_kernels(pd_ctx *c, int64_t n_steps, double *ms, int32_t *launches, int32_t n_out);

/* Streaming probe of known traffic (no context; for measuring the device's
 * achievable memory bandwidth and for scaling a profiler's byte counters):
 * mode 0 reads all `bytes` of src once (16-byte loads) and writes 4 bytes
 * per workgroup of its 4096 to dst (at least 16 KiB); mode 1 copies src to
 * dst.  Runs `reps` times back to back on the given stream (hipStream_t or
 * NULL) and returns the mean time per pass in *ms.  src, dst: device
 * buffers, 16-byte aligned; bytes a positive multiple of 16.
 * Errors: PD_E_INVALID (arguments), PD_E_DEVICE. */
pd_status pd_stream_probe(int32_t mode, const void *src, void *dst, int64_t bytes, int32_t reps,
                          void *hip_stream, double *ms);

/* Sizes: [0] nodes, [1] directed bonds, [2] padded bond slots, [3] cells,
 * [4] radix passes, [5] particles, [6] aggregates, [7] max LDS window,
 * [8] candidate-list rebuilds so far, [9] candidate slots per node. */
pd_status pd_sizes(const pd_ctx *c, int64_t out[10]);

/* Compaction observables at the current state (Sec. 7.4), per aggregate a,
 * out[12 a + k] (host buffer of 12 n_aggregates doubles):
 *   k = 0..7  force the particles exert on the left, right, floor and top wall
 *             (x, y each): minus the sum over the aggregate's nodes of each
 *             wall's share of the wall force of Sec. 4.5 (eq. wall-total),
 *             positions x + u, velocities v, top wall at t = step dt; a
 *             corner correction counts half for each of its two walls
 *   k = 8     volume fraction: sum of nodal areas / box area at time t
 *   k = 9, 10 broken and reference directed bonds (bulk damage = k9 / k10)
 *   k = 11    top-wall height at time t */
pd_status pd_observables(pd_ctx *c, double *out);
/* damage of each particle, broken / reference directed bonds of its nodes
 * (Sec. 3.1; 0 for a particle without bonds); host or device buffer of
 * n_particles doubles */
pd_status pd_particle_damage(pd_ctx *c, double *out, int32_t on_device);
/* Fragments (the child particles of Sec. 7.3): the connected components of
 * the graph of nodes joined by their intact bonds.  Bonds never join two
 * particles, so each component lies in one particle; a node that lost
 * every bond is a component of its own.  A bond joins its two nodes while
 * either of its directed copies is intact (the step breaks both together;
 * only pd_set_state can load copies that differ).  Reads the current bond
 * state only.
 *   label         N int32 (nullable): label[i] = smallest node index of
 *                 node i's component
 *   count         n_particles int32 (nullable): count[p] = components of
 *                 particle p with at least min_nodes nodes (min_nodes >= 1)
 *   n_components  (nullable) the number of all components
 * on_device = 1: label and count are device buffers on the library's
 * device, 0: host buffers.  Synchronous; the work is a few label rounds
 * (each a pass over the bond slots), bounded by N + 1. */
pd_status pd_fragments(pd_ctx *c, int32_t min_nodes, int32_t *label, int32_t *count,
                       int64_t *n_components, int32_t on_device);

/* ---------------------------------------------------------------------------
 * Learned modal closure (an extension: the paper has no reduced-order model).
 *
 * Particles that are rigid copies of one shape share that shape's modes: the
 * lowest K <= 32 non-rigid solutions of K phi = lambda M phi, K the
 * stiffness of the bond force of eq. (peri) linearised about the shape's
 * reference configuration, M = diag(rho V), phi^T M phi = 1.  A particle under
 * the closure is read in its best-fit rotated frame about its mass centroid
 * (weighted 2-D Procrustes); its modal amplitudes are q = Phi^T M u_body, its
 * internal force is M Phi g(q) rotated back, with g(q) = -lambda q (linear
 * closure) or -lambda q + sigma_r MLP(q / sigma_q) (learned closure: a
 * 32-256-256-32 SiLU network, bfloat16 weights, float32 accumulation on the
 * matrix cores), and it moves as a rigid body plus those modes: external
 * nodal forces (contact, walls) give its total force, its torque about the
 * centroid and the modal force Phi^T f_body, and the nodal accelerations are
 * rebuilt from them.  Gate, evaluated every step: a particle whose
 * first-order bound on its largest bond stretch, sum_k |q_k| sigma_k, passes
 * gate_frac * s0, or whose contact load sum_i |F_i| passes tau_c, returns to
 * the plain bond force from the next step on.  Every check_every steps (and at
 * pd_closure_check) all closure particles are checked against the plain bond
 * force at the current state: a particle whose largest true stretch passes
 * gate_frac * s0, or whose modal-force error passes err_tol times the larger
 * of |g_pd| and |lambda q|, returns to the plain bond force.  A particle never
 * re-enters the closure by itself (pd_closure_enable re-admits all).
 * The closure runs with candidate lists (tuning skin_factor > 0).
 * MLP parameters are packed float32 in the order W1 [256][32], b1 [256],
 * W2 [256][256], b2 [256], W3 [32][256], b3 [32] (weights [out][in]);
 * 82 464 values per shape.  Modes are [n_nodes][32][2] doubles (mode k of
 * node i, x then y), zero past the shape's mode count.
 * ------------------------------------------------------------------------- */
#define PD_CLOSURE_MODES 32
#define PD_CLOSURE_PARAMS 82464

/* shape_of_particle[n_particles]: shape id 0..S-1, or -1 (plain bond force
 * always).  Every particle of a shape must be a rigid copy of the shape's
 * first particle (same node count and order, same nodal masses); that first
 * particle's reference configuration defines the modes, computed here.
 * tau_c[S] (N/m) or NULL; an entry <= 0 takes 0.1 s0 E D (D the shape's
 * diameter).  Network parameters start at zero, i.e. the linear closure.
 * The closure starts switched off (pd_closure_enable).  PD_E_INVALID on a
 * particle that is not a copy of its shape, a shape with more than three
 * zero-stiffness modes, or more than 1024 nodes. */
pd_status pd_closure_setup(pd_ctx *c, const int32_t *shape_of_particle, double gate_frac,
                           const double *tau_c, int32_t check_every, double err_tol);
/* the shape's modes (host buffers, any may be NULL): n_nodes, mode count,
 * phi [n_nodes][32][2], lambda [32], sigma [32] (largest linear bond stretch
 * of each mode) */
pd_status pd_closure_modes(pd_ctx *c, int32_t shape, int32_t *n_nodes, int32_t *n_modes,
                           double *phi, double *lam, double *sig);
/* replace a shape's modes (host phi [n_nodes][32][2], lambda [32]); sigma is
 * recomputed */
pd_status pd_closure_set_modes(pd_ctx *c, int32_t shape, const double *phi, const double *lam);
/* network parameters (host, PD_CLOSURE_PARAMS floats) and the input/output
 * scales sigma_q, sigma_r [32] (either may be NULL: kept) */
pd_status pd_closure_load(pd_ctx *c, int32_t shape, const float *params, const float *sig_q,
                          const float *sig_r);
pd_status pd_closure_get(pd_ctx *c, int32_t shape, float *params, float *sig_q, float *sig_r);
/* 0: off (plain bond force everywhere); 1: linear closure; 2: learned
 * closure.  Switching on admits every closure particle; its state should lie
 * in its rigid + modal space (an undeformed particle does).
 *
 * mode | PD_CLOSURE_REDUCED (1 or 2 only): the reduced form.  A closure
 * particle's state is then its centroid, its rotation angle and its modal
 * amplitudes with their rates and accelerations (velocity Verlet on those:
 * centroid acceleration F/M + g, angular acceleration tau/I(q) with
 * I(q) = I0 + 2 b.q + q.q, b_k = sum m X.phi_k, modal acceleration
 * g(q) + Phi^T R(-phi) f), set at switch-on from the current nodes by the
 * same projections (mass centroid, best-fit angle, angular momentum and its
 * rate, modal projections of the body-frame deformation, velocity and
 * acceleration).  At each candidate-list rebuild the particle's active nodes
 * are listed: nodes with contact candidates, candidates of any node, and
 * nodes within the list radius of a wall.  A step computes contact and wall
 * forces for the active nodes only (the others cannot meet anything before
 * the next rebuild), reduces them with torque arms from the advanced nodal
 * positions, and reconstructs only the active nodes
 * (x + u = c + R(phi)(X + Phi q), velocity and acceleration by
 * differentiation); a bound on every node's motion since the rebuild,
 * |c - c_rb| + |phi - phi_rb| (r_max + sum |q_rb,k| phimax_k) +
 * sum |q_k - q_rb,k| phimax_k, against half the skin triggers the next
 * rebuild, and with a moving top wall the lists are rebuilt before it has
 * moved half the skin.  Every node is reconstructed before any call reads
 * the nodal state, and pd_set_state re-derives the reduced state from the
 * loaded nodes. */
#define PD_CLOSURE_REDUCED 4
pd_status pd_closure_enable(pd_ctx *c, int32_t mode);
/* Training snapshot at the current state, for every closure particle in the
 * order of pd_closure_particles: q [Pc][32] and the modal plain bond force
 * g = Phi^T R^T F_pd [Pc][32] (host or device buffers). */
pd_status pd_closure_snapshot(pd_ctx *c, double *q, double *g, int32_t on_device);
/* g = -lambda q + sigma_r MLP(q / sigma_q) for n rows q [n][32] of one shape */
pd_status pd_closure_forward(pd_ctx *c, int32_t shape, const double *q, double *g, int64_t n,
                             int32_t on_device);
/* loss and gradients (host buffers) of one batch: loss = mean over rows and
 * outputs of (MLP(q / sigma_q) - (g + lambda q) / sigma_r)^2; grads packed as
 * the parameters */
pd_status pd_closure_grads(pd_ctx *c, int32_t shape, const double *q, const double *g, int64_t n,
                           float *grads, double *loss);
/* train a shape's network on device data q, g [n][32] (samples of
 * pd_closure_snapshot): sigma_q, sigma_r from the data, Adam, batches drawn
 * with a counter-based generator from seed, step size lr with cosine decay
 * over the call; loss_out[iters] (host) or NULL.  A shape trained for the
 * first time starts from seeded uniform W1, W2 and zero W3 (the linear
 * closure). */
pd_status pd_closure_train(pd_ctx *c, int32_t shape, const double *q, const double *g, int64_t n,
                           int32_t iters, int32_t batch, double lr, uint64_t seed, float *loss_out);
/* a check against the plain bond force now (see above) */
pd_status pd_closure_check(pd_ctx *c);
/* out: closure particles, active now, fallbacks so far, checks so far, last
 * check's aggregate modal-force error sqrt(sum |g - g_pd|^2 / sum |g_pd|^2)
 * of the closure in use, the same for the linear closure, particles checked,
 * shapes */
pd_status pd_closure_stats(pd_ctx *c, double out[8]);
/* closure particles in snapshot order: particle index, shape, active flag */
pd_status pd_closure_particles(pd_ctx *c, int32_t *particle, int32_t *shape, int32_t *active);

#ifdef __cplusplus
}
#endif
#endif
