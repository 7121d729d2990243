/*
 * pd_oracle.h -- plain FP64 CPU oracle of the PeriDEM step (TEST INFRASTRUCTURE).
 *
 * This library exists only to check the GPU library: the tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it; the product path
 * never does.  It shares no code, header or constant with the GPU library.
 *
 * Method (Bhattacharya & Lipton, "Simulating grain shape effects and damage in
 * granular media using PeriDEM"):
 *   - bond-based peridynamic force with constant or conic micromodulus
 *     (Sec. 3, eq. (peri), eq. (pmb), Table tab:2d-peri), irreversible
 *     breaking when |s| > s0 and damage ratio (Sec. 3.1);
 *   - short-range repulsion (Sec. 4.1, eq. law-repulsive), regularized
 *     Coulomb friction (Sec. 4.2, eq. friction), normal damping (Sec. 4.3,
 *     eq. normal-damp), self-contact (Sec. 4.4);
 *   - analytic wall contact with corner correction (Sec. 4.5, eq.
 *     wall-repulsive, eq. wall-total);
 *   - velocity-Verlet time integration (Sec. 6.1, Algorithm alg:buildtree);
 *   - reference bonds restricted to segments inside the particle (Sec. 5),
 *     here by the plain definition (segment contained in the closed domain).
 * Readings of passages the paper leaves open are stated at the function that
 * applies them.
 */
#ifndef PD_ORACLE_H
#define PD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double rho, bulk_k, young_E, Gc, horizon;
    int32_t micro; /* 0 constant, 1 conic */
} or_material;

typedef struct {
    int32_t n_nodes, n_particles, n_aggregates, n_materials;
    const double *x, *y, *vol;
    const int32_t *particle_offset, *particle_material, *particle_aggregate;
    const or_material *materials;
    const int32_t *loop_offset, *loop_vertex_offset;
    const double *loop_xy;
    const double *u0x, *u0y, *v0x, *v0y; /* may be NULL (zero) */
    double contact_radius, friction_mu, damping_ratio;
    int32_t kn_mode; /* 0: K_n = c_w / R_c ; 1: K_n = 18 k / (pi eps^5) */
    const double *box;            /* [n_aggregates*4] xlo xhi ylo yhi at t = 0 */
    const double *top_wall_speed; /* [n_aggregates] downward speed, may be NULL */
    double gravity_x, gravity_y, dt;
    int32_t contact_mode; /* 0: brute force O(N^2); 1: bucket grid (same set, same sums) */
    int32_t n_threads;    /* OpenMP threads for the per-node loops (<=0: 1) */
} or_problem;

enum { OR_OK = 0, OR_E_INVALID = 1, OR_E_NOMEM = 2, OR_E_NONFINITE = 4, OR_E_ESCAPED = 5 };

/* force terms (force density F/V per node, Sec. 4.6 eq. full) */
enum { OR_T_PD = 1, OR_T_SELF = 2, OR_T_NBR = 4, OR_T_WALL = 8, OR_T_BODY = 16 };

typedef struct or_ctx or_ctx;

int or_create(const or_problem *p, or_ctx **out);
void or_destroy(or_ctx *c);
const char *or_error(const or_ctx *c);

/* per-material constants: out[m*4 + {0,1,2,3}] = c_w, s0, K_n, E */
int or_constants(const or_ctx *c, double *out);

/* reference bonds (CSR, columns ascending), directed */
int64_t or_n_bonds(const or_ctx *c);
int or_bonds(const or_ctx *c, int32_t *row /*[N+1]*/, int32_t *col /*[nnz]*/);

/* n steps of Algorithm alg:buildtree */
int or_step(or_ctx *c, int64_t n_steps);

/* force density by term at the current state (breaks not committed) */
int or_forces(or_ctx *c, uint32_t mask, double *fx, double *fy);

/* force the particles exert on each wall at the current state, per aggregate:
 * out[8 a + 2 w + k], w = left, right, floor, top, k = x, y (a corner
 * correction split evenly between its two walls); modifies the force buffers */
int or_wall_reactions(or_ctx *c, double *out);

/* damage ratio per node and number of broken directed bonds */
int or_damage(const or_ctx *c, double *phi, int64_t *n_broken_directed);

/* contact set at the current positions: unordered pairs i<j with
 * |p_i - p_j|^2 < R_c^2, sorted (i, then j). Returns the count; writes at most cap. */
int64_t or_contacts(or_ctx *c, int32_t *pi, int32_t *pj, int64_t cap);

/* state: u, v, a per node; broken flag per directed bond (CSR order); step index */
int or_get_state(const or_ctx *c, double *ux, double *uy, double *vx, double *vy,
                 double *ax, double *ay, uint8_t *broken, int64_t *step);
int or_set_state(or_ctx *c, const double *ux, const double *uy, const double *vx,
                 const double *vy, const double *ax, const double *ay,
                 const uint8_t *broken, int64_t step);

/* counters: [0] inter pairs, [1] self pairs, [2] stick, [3] slip, [4] wall regions,
 * [5] coincident pairs skipped, [6] bonds broken so far (directed) */
int or_counters(const or_ctx *c, int64_t out[8]);

/* geometry helper exposed for tests: 1 if the closed segment [a,b] lies in the
 * closed domain bounded by the particle's loops */
int or_segment_in_particle(const or_ctx *c, int32_t particle, double ax, double ay,
                           double bx, double by);

/* wall helpers exposed for tests: the regions of Sec. 4.5 by Gauss-Legendre
 * quadrature of their defining integrals (the printed closed forms pin them) */
void or_wall_segment(double Rc, double d, double *area, double *centroid_dist);
/* the intersection of the segments beyond two adjacent walls at signed
 * distances da, db and its first moments toward each wall */
void or_wall_corner(double Rc, double da, double db, double *area, double *Ix, double *Iy);
/* |S| (Rc - |c - p|) = integral over S of (Rc - x) dA, single wall at d */
double or_wall_segment_gap(double Rc, double d);

#ifdef __cplusplus
}
#endif
#endif
