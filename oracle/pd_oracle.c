/*
 * pd_oracle.c -- plain FP64 CPU oracle of the PeriDEM step (TEST INFRASTRUCTURE).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this file.  It is written for checking by eye against the paper, not
 * for speed: every sum runs over nodes in index order, contact pairs are
 * found by brute force (or by a bucket grid that visits the same candidates
 * in the same order), and reference bonds are filtered by the plain
 * definition of Sec. 5 (the closed segment must lie in the closed domain).
 *
 * Build: gcc -O2 -ffp-contract=off [-fopenmp] -shared -fPIC (no fast-math):
 * set-defining comparisons (bond inclusion, contact membership) use
 * r2 = dx*dx + dy*dy without fused multiply-add, as the GPU library does.
 */
#include "pd_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { T_PD = 0, T_SELF = 1, T_NBR = 2, T_WALL = 3, T_BODY = 4, NT = 5 };

struct or_ctx {
    int N, P, A, M;
    double *x, *y, *vol, *rho_n; /* per node */
    int *part;                   /* node -> particle */
    int *poff, *pmat, *pagg;
    or_material *mat;
    double *cw, *s0, *Kn, *E; /* per material */
    int *loff, *lvoff;
    double *lxy;
    double Rc, Rc2, mu, rd, dt, gx, gy;
    int kn_mode, contact_mode, nthreads;
    double *box, *vtop;
    /* bonds */
    int *row, *col;
    double *l0;
    uint8_t *broken, *brk_eval;
    int64_t nnz;
    /* state */
    double *ux, *uy, *vx, *vy, *ax, *ay, *px, *py;
    int64_t step;
    int status;
    /* nodal forces per term */
    double *F[NT][2];
    int64_t cnt[8];
    /* bucket grid */
    int *agg_cell0, *agg_ncx, *agg_ncy;
    double *agg_gx0, *agg_gy0, cell;
    int ncells;
    int *cell_head, *cell_next, *node_cell;
    char err[256];
};

static void set_err(or_ctx *c, const char *m) {
    if (c) snprintf(c->err, sizeof c->err, "%s", m);
}

const char *or_error(const or_ctx *c) { return c ? c->err : "null context"; }

/* ------------------------------------------------------------------------ */
/* constants: Table tab:2d-peri, Remark on nu = 1/3 in 2-D, Sec. 4.1 K_n      */
/* ------------------------------------------------------------------------ */
static void material_constants(const or_material *m, double Rc, int kn_mode, double *cw,
                               double *s0, double *Kn, double *E) {
    const double nu = 1.0 / 3.0; /* bond-based PD in 2-D (Remark after tab:2d-peri) */
    const double eps = m->horizon;
    /* E from the bulk modulus by the 2-D relation k = E / (2 (1 - nu)) unless given */
    const double Ey = m->young_E > 0.0 ? m->young_E : 2.0 * m->bulk_k * (1.0 - nu);
    if (m->micro == 0) { /* constant micromodulus */
        *cw = 6.0 * Ey / (M_PI * eps * eps * eps * (1.0 - nu));
        *s0 = sqrt(4.0 * M_PI * m->Gc / (9.0 * Ey * eps));
    } else { /* conic micromodulus w = 1 - |xi|/eps */
        *cw = 24.0 * Ey / (M_PI * eps * eps * eps * (1.0 - nu));
        *s0 = sqrt(5.0 * M_PI * m->Gc / (9.0 * Ey * eps));
    }
    if (kn_mode == 0)
        *Kn = *cw / Rc; /* self-contact and inter-particle laws coincide (Sec. 4.4, last remark) */
    else
        *Kn = 18.0 * m->bulk_k / (M_PI * eps * eps * eps * eps * eps); /* Sec. 4.1 as printed */
    *E = Ey;
}

int or_constants(const or_ctx *c, double *out) {
    for (int m = 0; m < c->M; ++m) {
        out[4 * m + 0] = c->cw[m];
        out[4 * m + 1] = c->s0[m];
        out[4 * m + 2] = c->Kn[m];
        out[4 * m + 3] = c->E[m];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5: a bond is kept iff the closed segment lies in the closed domain   */
/* ------------------------------------------------------------------------ */
/* coordinates relative to the particle's first node (the particle frame) */
static void frame_origin(const or_ctx *c, int p, double *rx, double *ry) {
    *rx = c->x[c->poff[p]];
    *ry = c->y[c->poff[p]];
}

/* point (mx, my), given in the particle frame, inside the closed domain */
static int point_in_closed_particle(const or_ctx *c, int p, double mx, double my, double tol) {
    double rx, ry;
    frame_origin(c, p, &rx, &ry);
    int inside = 0;
    for (int l = c->loff[p]; l < c->loff[p + 1]; ++l) {
        int v0 = c->lvoff[l], v1 = c->lvoff[l + 1], n = v1 - v0;
        for (int k = 0; k < n; ++k) {
            double Px = c->lxy[2 * (v0 + k)] - rx, Py = c->lxy[2 * (v0 + k) + 1] - ry;
            int kn = (k + 1 == n) ? 0 : k + 1;
            double Qx = c->lxy[2 * (v0 + kn)] - rx, Qy = c->lxy[2 * (v0 + kn) + 1] - ry;
            /* on the boundary (within tol) counts as inside */
            double ex = Qx - Px, ey = Qy - Py, L2 = ex * ex + ey * ey;
            double t = ((mx - Px) * ex + (my - Py) * ey) / L2;
            if (t < 0) t = 0;
            if (t > 1) t = 1;
            double qx = Px + t * ex - mx, qy = Py + t * ey - my;
            if (qx * qx + qy * qy <= tol * tol) return 1;
            if ((Py > my) != (Qy > my)) {
                double xint = Px + (my - Py) * (Qx - Px) / (Qy - Py);
                if (mx < xint) inside ^= 1;
            }
        }
    }
    return inside;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static int segment_in_particle(const or_ctx *c, int p, double ax, double ay, double bx,
                               double by, double *ts, double tol) {
    if (c->loff[p] == c->loff[p + 1]) return 1; /* no boundary loop given: convex */
    double ox, oy;
    frame_origin(c, p, &ox, &oy);
    ax -= ox;
    ay -= oy;
    bx -= ox;
    by -= oy;
    int nt = 0;
    ts[nt++] = 0.0;
    ts[nt++] = 1.0;
    const double rx = bx - ax, ry = by - ay;
    for (int l = c->loff[p]; l < c->loff[p + 1]; ++l) {
        int v0 = c->lvoff[l], v1 = c->lvoff[l + 1], n = v1 - v0;
        for (int k = 0; k < n; ++k) {
            double Px = c->lxy[2 * (v0 + k)] - ox, Py = c->lxy[2 * (v0 + k) + 1] - oy;
            int kn = (k + 1 == n) ? 0 : k + 1;
            double Qx = c->lxy[2 * (v0 + kn)] - ox, Qy = c->lxy[2 * (v0 + kn) + 1] - oy;
            double sx = Qx - Px, sy = Qy - Py, wx = Px - ax, wy = Py - ay;
            double den = rx * sy - ry * sx;
            if (den != 0.0) {
                double t = (wx * sy - wy * sx) / den;
                double u = (wx * ry - wy * rx) / den;
                if (t >= 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0) ts[nt++] = t;
            } else if (wx * ry - wy * rx == 0.0) { /* collinear: overlap end points */
                double rr = rx * rx + ry * ry;
                double t0 = (wx * rx + wy * ry) / rr;
                double t1 = ((Qx - ax) * rx + (Qy - ay) * ry) / rr;
                if (t0 >= 0.0 && t0 <= 1.0) ts[nt++] = t0;
                if (t1 >= 0.0 && t1 <= 1.0) ts[nt++] = t1;
            }
        }
    }
    qsort(ts, (size_t)nt, sizeof(double), cmp_double);
    for (int k = 0; k + 1 < nt; ++k) {
        if (!(ts[k + 1] > ts[k])) continue;
        double tm = 0.5 * (ts[k] + ts[k + 1]);
        if (!point_in_closed_particle(c, p, ax + tm * rx, ay + tm * ry, tol)) return 0;
    }
    return 1;
}

static double particle_tol(const or_ctx *c, int p) {
    /* 1e-12 of the particle's extent */
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int i = c->poff[p]; i < c->poff[p + 1]; ++i) {
        if (c->x[i] < xmin) xmin = c->x[i];
        if (c->x[i] > xmax) xmax = c->x[i];
        if (c->y[i] < ymin) ymin = c->y[i];
        if (c->y[i] > ymax) ymax = c->y[i];
    }
    double e = fmax(xmax - xmin, ymax - ymin);
    return 1e-12 * (e > 0 ? e : 1.0);
}

static int max_loop_edges(const or_ctx *c, int p) {
    int n = 0;
    for (int l = c->loff[p]; l < c->loff[p + 1]; ++l) n += c->lvoff[l + 1] - c->lvoff[l];
    return n;
}

int or_segment_in_particle(const or_ctx *c, int32_t p, double ax, double ay, double bx,
                           double by) {
    int ne = max_loop_edges(c, p);
    double *ts = (double *)malloc(sizeof(double) * (size_t)(2 * ne + 4));
    int r = segment_in_particle(c, p, ax, ay, bx, by, ts, particle_tol(c, p));
    free(ts);
    return r;
}

/* Algorithm alg:buildtree, reference neighbours: x' in the same particle with
 * |x' - x| < eps, minus non-bonds (Sec. 5).  The strict inequality is taken
 * against (eps - 1e-9 eps)^2 so that lattice distances equal to eps are
 * excluded robustly; r2 is dx*dx + dy*dy without contraction. */
static int build_bonds(or_ctx *c) {
    int N = c->N;
    c->row = (int *)calloc((size_t)N + 1, sizeof(int));
    if (!c->row) return OR_E_NOMEM;
    /* pass 1: count; pass 2: fill */
    int64_t cap = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t nnz = 0;
        for (int p = 0; p < c->P; ++p) {
            const or_material *m = &c->mat[c->pmat[p]];
            const double thr = m->horizon - 1e-9 * m->horizon;
            const double thr2 = thr * thr;
            int ne = max_loop_edges(c, p);
            double *ts = (double *)malloc(sizeof(double) * (size_t)(2 * ne + 4));
            double tol = particle_tol(c, p);
            for (int i = c->poff[p]; i < c->poff[p + 1]; ++i) {
                if (pass == 1) c->row[i] = (int)nnz;
                for (int j = c->poff[p]; j < c->poff[p + 1]; ++j) {
                    if (j == i) continue;
                    double dx = c->x[j] - c->x[i], dy = c->y[j] - c->y[i];
                    double d2 = dx * dx + dy * dy;
                    if (!(d2 < thr2)) continue;
                    if (!segment_in_particle(c, p, c->x[i], c->y[i], c->x[j], c->y[j], ts, tol))
                        continue;
                    if (pass == 1) {
                        c->col[nnz] = j;
                        c->l0[nnz] = sqrt(d2);
                    }
                    ++nnz;
                }
            }
            free(ts);
        }
        if (pass == 0) {
            cap = nnz;
            c->col = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
            c->l0 = (double *)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
            c->broken = (uint8_t *)calloc((size_t)(cap > 0 ? cap : 1), 1);
            c->brk_eval = (uint8_t *)calloc((size_t)(cap > 0 ? cap : 1), 1);
            if (!c->col || !c->l0 || !c->broken || !c->brk_eval) return OR_E_NOMEM;
        } else {
            c->row[N] = (int)nnz;
            c->nnz = nnz;
        }
    }
    return OR_OK;
}

int64_t or_n_bonds(const or_ctx *c) { return c->nnz; }

int or_bonds(const or_ctx *c, int32_t *row, int32_t *col) {
    memcpy(row, c->row, sizeof(int) * ((size_t)c->N + 1));
    memcpy(col, c->col, sizeof(int) * (size_t)c->nnz);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* bucket grid: only a way to visit candidates; the set is the brute one     */
/* ------------------------------------------------------------------------ */
static void setup_grid(or_ctx *c) {
    /* cell side >= R_c; coarser when the boxes are huge compared with the
     * node count (only the visiting cost changes, never the set) */
    double area = 0.0;
    for (int a = 0; a < c->A; ++a)
        area += (c->box[4 * a + 1] - c->box[4 * a] + 4 * c->Rc) *
                (c->box[4 * a + 3] - c->box[4 * a + 2] + 4 * c->Rc);
    c->cell = c->Rc;
    double maxcells = 16.0 * (double)c->N + 4096.0;
    if (area / (c->cell * c->cell) > maxcells) c->cell = sqrt(area / maxcells);
    c->agg_cell0 = (int *)malloc(sizeof(int) * (size_t)c->A);
    c->agg_ncx = (int *)malloc(sizeof(int) * (size_t)c->A);
    c->agg_ncy = (int *)malloc(sizeof(int) * (size_t)c->A);
    c->agg_gx0 = (double *)malloc(sizeof(double) * (size_t)c->A);
    c->agg_gy0 = (double *)malloc(sizeof(double) * (size_t)c->A);
    int nc = 0;
    for (int a = 0; a < c->A; ++a) {
        double xlo = c->box[4 * a], xhi = c->box[4 * a + 1], ylo = c->box[4 * a + 2],
               yhi = c->box[4 * a + 3];
        c->agg_gx0[a] = xlo - 2 * c->cell;
        c->agg_gy0[a] = ylo - 2 * c->cell;
        (void)yhi;
        c->agg_ncx[a] = (int)((xhi - xlo) / c->cell) + 5;
        c->agg_ncy[a] = (int)((yhi - ylo) / c->cell) + 5;
        c->agg_cell0[a] = nc;
        nc += c->agg_ncx[a] * c->agg_ncy[a];
    }
    c->ncells = nc;
    c->cell_head = (int *)malloc(sizeof(int) * (size_t)nc);
    c->cell_next = (int *)malloc(sizeof(int) * (size_t)c->N);
    c->node_cell = (int *)malloc(sizeof(int) * (size_t)c->N * 2);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void fill_grid(or_ctx *c) {
    for (int k = 0; k < c->ncells; ++k) c->cell_head[k] = -1;
    for (int i = c->N - 1; i >= 0; --i) { /* reverse so that lists run in index order */
        int a = c->pagg[c->part[i]];
        int cx = clampi((int)floor((c->px[i] - c->agg_gx0[a]) / c->cell), 0, c->agg_ncx[a] - 1);
        int cy = clampi((int)floor((c->py[i] - c->agg_gy0[a]) / c->cell), 0, c->agg_ncy[a] - 1);
        c->node_cell[2 * i] = cx;
        c->node_cell[2 * i + 1] = cy;
        int id = c->agg_cell0[a] + cy * c->agg_ncx[a] + cx;
        c->cell_next[i] = c->cell_head[id];
        c->cell_head[id] = i;
    }
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* candidates j != i of node i, ascending; returns the count */
static int candidates(const or_ctx *c, int i, int *buf, int cap) {
    int n = 0;
    int a = c->pagg[c->part[i]];
    if (c->contact_mode == 0) {
        for (int j = 0; j < c->N; ++j)
            if (j != i && c->pagg[c->part[j]] == a) {
                if (n < cap) buf[n] = j;
                ++n;
            }
        return n;
    }
    int cx = c->node_cell[2 * i], cy = c->node_cell[2 * i + 1];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int x = cx + dx, y = cy + dy;
            if (x < 0 || y < 0 || x >= c->agg_ncx[a] || y >= c->agg_ncy[a]) continue;
            for (int j = c->cell_head[c->agg_cell0[a] + y * c->agg_ncx[a] + x]; j >= 0;
                 j = c->cell_next[j])
                if (j != i) {
                    if (n < cap) buf[n] = j;
                    ++n;
                }
        }
    if (n <= cap) qsort(buf, (size_t)n, sizeof(int), cmp_int);
    return n;
}

/* ------------------------------------------------------------------------ */
/* force laws                                                                */
/* ------------------------------------------------------------------------ */
static int bond_intact(const or_ctx *c, int i, int j) {
    /* binary search of j in the (ascending) CSR row of i */
    int lo = c->row[i], hi = c->row[i + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        if (c->col[mid] == j) return !c->broken[mid];
        if (c->col[mid] < j)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0; /* no reference bond (outside the horizon or a filtered non-bond) */
}

/* Damping (Sec. 4.3) and friction (Sec. 4.2) of a contact on node i.
 * e: unit normal from i toward the partner; (vrx, vry) = v_i - v_partner;
 * Frmag = |F_r|; Kd = stiffness used in beta_d; Vp = partner volume (or wall
 * segment area).  Readings: damping force -c (v.e) e with
 * c = 2 r_d sqrt(Kd rho_i V_i^2 V_p) (dissipative, Kelvin-Voigt equivalence);
 * friction opposes the tangential part of v_i - v_partner. */
static void damp_friction(const or_ctx *c, double rho_i, double Vi, double Vp, double Kd,
                          double ex, double ey, double vrx, double vry, double Frmag,
                          double *fx, double *fy, int64_t *stick, int64_t *slip) {
    double vn = vrx * ex + vry * ey;
    double cd = 2.0 * c->rd * sqrt(Kd * rho_i * Vi * Vi * Vp);
    double Fdx = -cd * vn * ex, Fdy = -cd * vn * ey;
    double vtx = vrx - vn * ex, vty = vry - vn * ey;
    double vt = sqrt(vtx * vtx + vty * vty);
    double vthr = c->mu * Frmag * c->dt / (rho_i * Vi);
    double Ffx, Ffy;
    if (vt > vthr) { /* slip: magnitude mu |F_r| against the tangential relative velocity */
        Ffx = -c->mu * Frmag * vtx / vt;
        Ffy = -c->mu * Frmag * vty / vt;
        ++*slip;
    } else { /* stick: regularized, eps_f = dt / (rho V_i) */
        Ffx = -(rho_i * Vi / c->dt) * vtx;
        Ffy = -(rho_i * Vi / c->dt) * vty;
        ++*stick;
    }
    *fx = Fdx + Ffx;
    *fy = Fdy + Ffy;
}

/* contact forces on node i (inter-particle and self-contact), one-sided */
static void contact_node(or_ctx *c, int i, const double *vx, const double *vy, int *buf,
                         int cap, int64_t *cnt) {
    const int pi = c->part[i];
    const int mi = c->pmat[pi];
    const double Vi = c->vol[i], rho_i = c->rho_n[i];
    double fsx = 0, fsy = 0, fnx = 0, fny = 0;
    int n = candidates(c, i, buf, cap);
    if (n > cap) n = cap; /* cap is N: never hit */
    for (int q = 0; q < n; ++q) {
        int j = buf[q];
        double dx = c->px[j] - c->px[i], dy = c->py[j] - c->py[i];
        double r2 = dx * dx + dy * dy;
        if (!(r2 < c->Rc2)) continue;
        if (r2 == 0.0) { /* coincident nodes: no direction; skipped and counted */
            ++cnt[5];
            continue;
        }
        const int pj = c->part[j];
        const int same = (pj == pi);
        if (same && bond_intact(c, i, j)) continue; /* the bond acts, not contact */
        const double d = sqrt(r2);
        const double ex = dx / d, ey = dy / d;
        const double Vj = c->vol[j];
        double coef, Kd;
        if (!same) {
            const int mj = c->pmat[pj];
            const double Ka = c->Kn[mi], Kb = c->Kn[mj];
            const double Kn = (2.0 * Ka * Kb) / (Ka + Kb); /* harmonic mean, Sec. 4.1 */
            coef = -Kn * (c->Rc - d);                      /* F_r = coef V_i V_j e */
            Kd = Kn;
            ++cnt[0];
        } else {
            const double cw = c->cw[mi];
            const double X = c->x[j] - c->x[i], Y = c->y[j] - c->y[i];
            const double L = sqrt(X * X + Y * Y); /* reference distance |xi| */
            if (L < c->Rc)
                coef = (d < L) ? cw * (d - L) / L : 0.0;
            else
                coef = cw * (d - c->Rc) / c->Rc;
            Kd = cw / c->Rc;
            ++cnt[1];
        }
        const double Frx = coef * Vi * Vj * ex, Fry = coef * Vi * Vj * ey;
        const double Frmag = fabs(coef) * Vi * Vj;
        double fdx, fdy;
        damp_friction(c, rho_i, Vi, Vj, Kd, ex, ey, vx[i] - vx[j], vy[i] - vy[j], Frmag, &fdx,
                      &fdy, &cnt[2], &cnt[3]);
        if (same) {
            fsx += Frx + fdx;
            fsy += Fry + fdy;
        } else {
            fnx += Frx + fdx;
            fny += Fry + fdy;
        }
    }
    c->F[T_SELF][0][i] = fsx;
    c->F[T_SELF][1][i] = fsy;
    c->F[T_NBR][0][i] = fnx;
    c->F[T_NBR][1][i] = fny;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.5 wall regions by quadrature of their defining integrals           */
/* ------------------------------------------------------------------------ */
/* The regions are parts of the contact disk of radius Rc about the node: the
 * circular segment beyond one wall and the intersection of two such segments
 * at a corner.  Their areas and first moments are integrals over the region,
 * evaluated here by Gauss-Legendre quadrature on vertical strips: in the
 * frame of the node with the wall (or the two walls) beyond x = da (and
 * y = db), a strip at abscissa x = Rc cos(theta) runs from its lower end
 * (the line y = db, or the circle) to the circle y = Rc sin(theta), and
 * dx = Rc sin(theta) dtheta.  The integrands are smooth in theta, so a
 * 20-point rule is exact to rounding; each panel is checked against its two
 * halves and halved until they agree to 1e-15. */
#define GL_N 20
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;

/* nodes and weights of the n-point Gauss-Legendre rule on [-1, 1]: roots of
 * the Legendre polynomial P_n by Newton's method (P_n and P_n' from the
 * three-term recurrence), weights 2 / ((1 - x^2) P_n'(x)^2) */
static void gl_init(void) {
    if (gl_ready) return;
    const int n = GL_N;
    for (int k = 0; k < n; ++k) {
        double x = cos(M_PI * (k + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        gl_x[k] = x;
        gl_w[k] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

/* the strip integrands at angle theta (abscissa x = Rc cos theta, top
 * Rc sin theta), times dx/dtheta: area, moment along x, moment along y, and
 * the integral of (Rc - x), with Rc - x = 2 Rc sin^2(theta/2) */
#define NQ 4
typedef struct {
    double Rc, db;
    int circle; /* lower end: 0 the line y = db, 1 the circle y = -Rc sin theta */
} strip_args;

/* out[NQ..2NQ-1]: the same products with |top| + |bot| for the strip's
 * length and absolute values elsewhere, the scale of their rounding errors
 * (top - bot and top + bot cancel where the strip is short or its ends are
 * nearly opposite) */
static void strip(const strip_args *s, double th, double out[2 * NQ]) {
    const double R = s->Rc;
    const double sn = sin(th), x = R * cos(th), top = R * sn, sh = sin(0.5 * th);
    const double bot = s->circle ? -top : s->db;
    const double jac = R * sn; /* dx / dtheta */
    const double len = top - bot;
    out[0] = len * jac;
    out[1] = x * len * jac;
    out[2] = 0.5 * (top - bot) * (top + bot) * jac;
    out[3] = 2.0 * R * sh * sh * len * jac;
    const double span = fabs(top) + fabs(bot); /* |len| before cancellation */
    out[NQ + 0] = span * fabs(jac);
    out[NQ + 1] = fabs(x) * span * fabs(jac);
    out[NQ + 2] = 0.5 * span * span * fabs(jac);
    out[NQ + 3] = 2.0 * R * sh * sh * span * fabs(jac);
}

/* the rule on one panel: integrals out[0..NQ-1] and the integrals of the
 * absolute products out[NQ..2NQ-1] */
static void gl_panel(const strip_args *s, double a, double b, double out[2 * NQ]) {
    const double m = 0.5 * (a + b), r = 0.5 * (b - a);
    for (int q = 0; q < 2 * NQ; ++q) out[q] = 0.0;
    for (int k = 0; k < GL_N; ++k) {
        double f[2 * NQ];
        strip(s, m + r * gl_x[k], f);
        for (int q = 0; q < 2 * NQ; ++q) out[q] += gl_w[k] * f[q];
    }
    for (int q = 0; q < 2 * NQ; ++q) out[q] *= r;
}

/* the panel [a, b] whose one-panel value is `whole`: accepted when its two
 * halves agree with it to 1e-13 of the integral of the absolute products,
 * else each half in turn (at most 8 halvings).  The integrands are smooth,
 * so the 20-point rule is exact to rounding on any panel here; the two
 * evaluations then differ only by the rounding of the abscissae (sin theta
 * near 0 or pi magnifies it by |cot theta|), far below this bound. */
static void gl_adapt(const strip_args *s, double a, double b, const double whole[2 * NQ],
                     int depth, double out[NQ]) {
    const double m = 0.5 * (a + b);
    double l[2 * NQ], r[2 * NQ];
    gl_panel(s, a, m, l);
    gl_panel(s, m, b, r);
    int ok = 1;
    for (int q = 0; q < NQ; ++q)
        if (fabs((l[q] + r[q]) - whole[q]) > 1e-13 * (l[NQ + q] + r[NQ + q])) ok = 0;
    if (ok || depth >= 8) {
        for (int q = 0; q < NQ; ++q) out[q] = l[q] + r[q];
        return;
    }
    double lo[NQ], hi[NQ];
    gl_adapt(s, a, m, l, depth + 1, lo);
    gl_adapt(s, m, b, r, depth + 1, hi);
    for (int q = 0; q < NQ; ++q) out[q] = lo[q] + hi[q];
}

/* adds the strips of angles [a, b] (0 <= a <= b <= pi) to acc */
static void strips(double Rc, double db, int circle, double a, double b, double acc[NQ]) {
    if (!(b > a)) return;
    gl_init();
    const strip_args s = {Rc, db, circle};
    double whole[2 * NQ], out[NQ];
    gl_panel(&s, a, b, whole);
    gl_adapt(&s, a, b, whole, 0, out);
    for (int q = 0; q < NQ; ++q) acc[q] += out[q];
}

/* angle theta in [0, pi] of the abscissa x = Rc cos(theta), from
 * 1 - cos(theta) = 2 sin^2(theta/2): well conditioned as x -> Rc */
static double theta_of(double Rc, double x) { return 2.0 * asin(sqrt((Rc - x) / (2.0 * Rc))); }

/* Region {x > da, y > db, x^2 + y^2 < Rc^2} (a corner; db <= -Rc: the
 * segment beyond x = da alone): area and first moments about the node. */
static void region_integrals(double Rc, double da, double db, double acc[NQ]) {
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const double tda = theta_of(Rc, da); /* strips x in (da, Rc): theta in [0, tda) */
    if (db <= -Rc) {                     /* no lower wall: whole chords */
        strips(Rc, 0.0, 1, 0.0, tda, acc);
    } else if (db >= 0.0) {
        /* the line y = db is the lower end where the circle is above it:
         * sin(theta) > db / Rc */
        const double tb = asin(db / Rc);
        strips(Rc, db, 0, tb, fmin(tda, M_PI - tb), acc);
    } else {
        /* the line is the lower end where it lies above the lower circle,
         * sin(theta) > -db / Rc; whole chords elsewhere */
        const double tc = asin(-db / Rc);
        strips(Rc, db, 1, 0.0, fmin(tc, tda), acc);
        strips(Rc, db, 0, tc, fmin(tda, M_PI - tc), acc);
        strips(Rc, db, 1, M_PI - tc, tda, acc);
    }
}

/* Sec. 4.5: circular segment of the contact disk beyond one wall at signed
 * distance d (-Rc < d < Rc): its area |S| and the distance of its centroid
 * from the node (the printed closed forms are the pins of these integrals) */
void or_wall_segment(double Rc, double d, double *area, double *centroid_dist) {
    double q[NQ];
    region_integrals(Rc, d, -2.0 * Rc, q);
    *area = q[0];
    *centroid_dist = q[0] > 0.0 ? q[1] / q[0] : Rc;
}

/* |S| (Rc - |c - p|) = integral over S of (Rc - x) dA: the factor of the
 * single-wall repulsion (Sec. 4.5), whose integrand is positive, so that it
 * keeps its precision as d -> Rc, where |S| and Rc - |c - p| both vanish */
double or_wall_segment_gap(double Rc, double d) {
    double q[NQ];
    region_integrals(Rc, d, -2.0 * Rc, q);
    return q[3];
}

/* Sec. 4.5: the part of the contact disk beyond two adjacent walls at signed
 * distances da, db (the intersection of the two segments), and its first
 * moments Ix (toward wall a) and Iy (toward wall b) about the node */
void or_wall_corner(double Rc, double da, double db, double *area, double *Ix, double *Iy) {
    double q[NQ];
    region_integrals(Rc, da, db, q);
    *area = q[0];
    *Ix = q[1];
    *Iy = q[2];
}

/* one wall region (segment or corner) acting on node i: repulsion of
 * magnitude Frmag along -e (e points from the node toward the region's
 * centroid), damping and friction against the region's velocity (wvx, wvy);
 * the region's area A stands for the partner volume */
static void wall_region(const or_ctx *c, int i, double Kn, double A, double Frmag, double ex,
                        double ey, double wvx, double wvy, const double *vx, const double *vy,
                        double sign, double *fx, double *fy, int64_t *cnt) {
    const double Vi = c->vol[i], rho_i = c->rho_n[i];
    const double Frx = -Frmag * ex, Fry = -Frmag * ey;
    double fdx, fdy;
    damp_friction(c, rho_i, Vi, A, Kn, ex, ey, vx[i] - wvx, vy[i] - wvy, fabs(Frmag), &fdx, &fdy,
                  &cnt[2], &cnt[3]);
    *fx += sign * (Frx + fdx);
    *fy += sign * (Fry + fdy);
    ++cnt[4];
}

/* walls of node i: left, right, floor, top (top at height yhi0 - v t).
 * With split != NULL, also each wall's share of the force on the node:
 * split[2 w], split[2 w + 1] for wall w; a wall segment counts for its wall,
 * a corner correction half for each of its two walls. */
static int wall_node_split(or_ctx *c, int i, double t, const double *vx, const double *vy,
                           int64_t *cnt, double *split) {
    const int a = c->pagg[c->part[i]];
    const double Rc = c->Rc;
    const double xlo = c->box[4 * a], xhi = c->box[4 * a + 1], ylo = c->box[4 * a + 2];
    const double vtop = c->vtop ? c->vtop[a] : 0.0;
    const double yhi = c->box[4 * a + 3] - vtop * t;
    /* signed inward distances and unit normals toward each wall */
    const double d[4] = {c->px[i] - xlo, xhi - c->px[i], c->py[i] - ylo, yhi - c->py[i]};
    const double nx[4] = {-1.0, 1.0, 0.0, 0.0}, ny[4] = {0.0, 0.0, -1.0, 1.0};
    const double wv[4] = {0.0, 0.0, 0.0, -vtop}; /* wall velocity (y component) */
    const double Kn = c->Kn[c->pmat[c->part[i]]];
    double fx = 0.0, fy = 0.0;
    int st = OR_OK;
    for (int w = 0; w < 4; ++w) {
        if (!(d[w] > -Rc)) st = OR_E_ESCAPED;
        if (d[w] < Rc && d[w] > -Rc) {
            /* F = -K_n (Rc - |c_l - p|) V_i |S_l| e_l, with |S_l| (Rc - |c_l - p|)
             * the integral of (Rc - x) over S_l (no cancellation as d -> Rc) */
            double q[NQ];
            region_integrals(Rc, d[w], -2.0 * Rc, q);
            const double A = q[0];
            const double Frmag = Kn * c->vol[i] * q[3];
            if (A > 0.0) {
                double rx = 0.0, ry = 0.0;
                wall_region(c, i, Kn, A, Frmag, nx[w], ny[w], 0.0, wv[w], vx, vy, +1.0, &rx, &ry,
                            cnt);
                fx += rx;
                fy += ry;
                if (split) {
                    split[2 * w] += rx;
                    split[2 * w + 1] += ry;
                }
            }
        }
    }
    /* adjacent pairs: (left, floor), (floor, right), (right, top), (top, left) */
    static const int pa[4] = {0, 2, 1, 3}, pb[4] = {2, 1, 3, 0};
    for (int k = 0; k < 4; ++k) {
        int wa = pa[k], wb = pb[k];
        double da = d[wa], db = d[wb];
        /* S_a and S_b overlap iff the point of the quadrant beyond both
         * walls nearest to the node lies within Rc (for da, db >= 0 the
         * printed condition da^2 + db^2 < Rc^2) */
        const double qa = da > 0.0 ? da : 0.0, qb = db > 0.0 ? db : 0.0;
        if (da > -Rc && db > -Rc && qa * qa + qb * qb < Rc * Rc) {
            double A, Ix, Iy;
            or_wall_corner(Rc, da, db, &A, &Ix, &Iy);
            if (!(A > 0.0)) continue;
            double cx = (Ix * nx[wa] + Iy * nx[wb]) / A, cy = (Ix * ny[wa] + Iy * ny[wb]) / A;
            double dist = sqrt(cx * cx + cy * cy);
            double ex = cx / dist, ey = cy / dist;
            /* corner region moves with the top wall when it borders it */
            double wvy = (wa == 3 || wb == 3) ? -vtop : 0.0;
            const double Frmag = Kn * (Rc - dist) * c->vol[i] * A;
            double rx = 0.0, ry = 0.0;
            wall_region(c, i, Kn, A, Frmag, ex, ey, 0.0, wvy, vx, vy, -1.0, &rx, &ry, cnt);
            fx += rx;
            fy += ry;
            if (split) {
                split[2 * wa] += 0.5 * rx;
                split[2 * wa + 1] += 0.5 * ry;
                split[2 * wb] += 0.5 * rx;
                split[2 * wb + 1] += 0.5 * ry;
            }
        }
    }
    c->F[T_WALL][0][i] = fx;
    c->F[T_WALL][1][i] = fy;
    return st;
}

static int wall_node(or_ctx *c, int i, double t, const double *vx, const double *vy,
                     int64_t *cnt) {
    return wall_node_split(c, i, t, vx, vy, cnt, NULL);
}

/* PD force on node i (eq. peri, eq. pmb); bonds with |s| > s0 carry no force
 * and are flagged in brk_eval (committed by the caller during a step) */
static void pd_node(or_ctx *c, int i) {
    const int p = c->part[i];
    const int m = c->pmat[p];
    const double cw = c->cw[m], s0 = c->s0[m], eps = c->mat[m].horizon;
    const int conic = c->mat[m].micro == 1;
    const double Vi = c->vol[i];
    double fx = 0.0, fy = 0.0;
    for (int k = c->row[i]; k < c->row[i + 1]; ++k) {
        c->brk_eval[k] = 0;
        if (c->broken[k]) continue;
        const int j = c->col[k];
        /* bond xi = x' - x, relative displacement eta = u' - u (Sec. 3) */
        const double X = c->x[j] - c->x[i], Y = c->y[j] - c->y[i];
        const double ex = c->ux[j] - c->ux[i], ey = c->uy[j] - c->uy[i];
        const double dx = X + ex, dy = Y + ey; /* xi + eta */
        const double l = sqrt(dx * dx + dy * dy);
        const double L0 = c->l0[k]; /* |xi| */
        /* s = (|xi + eta| - |xi|) / |xi|, evaluated as
         *     eta . (xi + eta + xi) / (|xi| (|xi + eta| + |xi|)),
         * the same quantity without the cancellation of |xi + eta| - |xi| at
         * small strain (both evaluations of a bond give the same bits from its
         * two ends: every factor flips sign exactly) */
        const double s = (ex * (dx + X) + ey * (dy + Y)) / (L0 * (l + L0));
        if (fabs(s) > s0) { /* Sec. 3.1: broken when |s| exceeds s0 */
            c->brk_eval[k] = 1;
            continue;
        }
        const double w = conic ? 1.0 - L0 / eps : 1.0;
        const double f = cw * w * s * Vi * c->vol[j]; /* nodal force magnitude */
        fx += f * dx / l;
        fy += f * dy / l;
    }
    c->F[T_PD][0][i] = fx;
    c->F[T_PD][1][i] = fy;
}

/* all terms at positions p = x + u, velocities (vx, vy), wall time t */
static int eval_forces(or_ctx *c, const double *vx, const double *vy, double t) {
    const int N = c->N;
    for (int i = 0; i < N; ++i) {
        c->px[i] = c->x[i] + c->ux[i];
        c->py[i] = c->y[i] + c->uy[i];
    }
    if (c->contact_mode == 1) fill_grid(c);
    int st = OR_OK;
    int64_t cnt[8] = {0};
    int nth = c->nthreads > 0 ? c->nthreads : 1;
    (void)nth;
#pragma omp parallel num_threads(nth) reduction(+ : cnt[:8])
    {
        int *buf = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
        int stl = OR_OK;
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) {
            /* contact first: self-contact sees bonds intact at the start of the step */
            contact_node(c, i, vx, vy, buf, N, cnt);
            int s = wall_node(c, i, t, vx, vy, cnt);
            if (s != OR_OK) stl = s;
        }
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i) pd_node(c, i);
        free(buf);
#pragma omp critical
        if (stl != OR_OK) st = stl;
    }
    for (int k = 0; k < 8; ++k) c->cnt[k] += cnt[k];
    for (int i = 0; i < N; ++i) {
        const double m = c->rho_n[i] * c->vol[i];
        c->F[T_BODY][0][i] = m * c->gx;
        c->F[T_BODY][1][i] = m * c->gy;
    }
    return st;
}

static int check_finite(const or_ctx *c) {
    for (int i = 0; i < c->N; ++i)
        if (!isfinite(c->ux[i]) || !isfinite(c->uy[i]) || !isfinite(c->vx[i]) ||
            !isfinite(c->vy[i]))
            return OR_E_NONFINITE;
    return OR_OK;
}

/* acceleration from the summed nodal force: a = F / (rho V) + g */
static void accel_from_forces(or_ctx *c, double *ax, double *ay) {
    for (int i = 0; i < c->N; ++i) {
        const double Fx = c->F[T_PD][0][i] + c->F[T_SELF][0][i] + c->F[T_NBR][0][i] +
                          c->F[T_WALL][0][i];
        const double Fy = c->F[T_PD][1][i] + c->F[T_SELF][1][i] + c->F[T_NBR][1][i] +
                          c->F[T_WALL][1][i];
        const double m = c->rho_n[i] * c->vol[i];
        ax[i] = Fx / m + c->gx;
        ay[i] = Fy / m + c->gy;
    }
}

static void commit_breaks(or_ctx *c) {
    for (int64_t k = 0; k < c->nnz; ++k)
        if (c->brk_eval[k]) {
            c->broken[k] = 1;
            ++c->cnt[6];
        }
}

/* ------------------------------------------------------------------------ */
/* setup                                                                     */
/* ------------------------------------------------------------------------ */
static void *dup(const void *p, size_t n) {
    void *q = malloc(n > 0 ? n : 1);
    if (q && p && n) memcpy(q, p, n);
    return q;
}

int or_create(const or_problem *p, or_ctx **out) {
    gl_init(); /* the quadrature rule, before any parallel region reads it */
    *out = NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    if (!c) return OR_E_NOMEM;
    *out = c;
    if (p->n_nodes < 0 || p->n_particles < 1 || p->n_materials < 1 || !(p->dt > 0) ||
        !(p->contact_radius > 0)) {
        set_err(c, "invalid sizes, dt or contact radius");
        return OR_E_INVALID;
    }
    const int N = p->n_nodes, P = p->n_particles, M = p->n_materials;
    const int A = p->n_aggregates > 0 ? p->n_aggregates : 1;
    c->N = N;
    c->P = P;
    c->A = A;
    c->M = M;
    c->x = (double *)dup(p->x, sizeof(double) * N);
    c->y = (double *)dup(p->y, sizeof(double) * N);
    c->vol = (double *)dup(p->vol, sizeof(double) * N);
    c->poff = (int *)dup(p->particle_offset, sizeof(int) * (P + 1));
    c->pmat = (int *)dup(p->particle_material, sizeof(int) * P);
    c->pagg = (int *)calloc((size_t)P, sizeof(int));
    if (p->particle_aggregate) memcpy(c->pagg, p->particle_aggregate, sizeof(int) * P);
    c->mat = (or_material *)dup(p->materials, sizeof(or_material) * M);
    c->loff = (int *)dup(p->loop_offset, sizeof(int) * (P + 1));
    int nl = c->loff[P];
    c->lvoff = (int *)dup(p->loop_vertex_offset, sizeof(int) * (nl + 1));
    int nv = c->lvoff[nl];
    c->lxy = (double *)dup(p->loop_xy, sizeof(double) * 2 * nv);
    c->box = (double *)dup(p->box, sizeof(double) * 4 * A);
    c->vtop = p->top_wall_speed ? (double *)dup(p->top_wall_speed, sizeof(double) * A) : NULL;
    c->Rc = p->contact_radius;
    c->Rc2 = p->contact_radius * p->contact_radius;
    c->mu = p->friction_mu;
    c->rd = p->damping_ratio;
    c->dt = p->dt;
    c->gx = p->gravity_x;
    c->gy = p->gravity_y;
    c->kn_mode = p->kn_mode;
    c->contact_mode = p->contact_mode;
    c->nthreads = p->n_threads;
    for (int q = 0; q < P; ++q)
        if (c->poff[q + 1] <= c->poff[q] || c->pmat[q] < 0 || c->pmat[q] >= M ||
            c->pagg[q] < 0 || c->pagg[q] >= A) {
            set_err(c, "bad particle offsets, material or aggregate");
            return OR_E_INVALID;
        }
    if (c->poff[0] != 0 || c->poff[P] != N) {
        set_err(c, "particle offsets must cover all nodes");
        return OR_E_INVALID;
    }
    c->part = (int *)malloc(sizeof(int) * (size_t)N);
    c->rho_n = (double *)malloc(sizeof(double) * (size_t)N);
    for (int q = 0; q < P; ++q)
        for (int i = c->poff[q]; i < c->poff[q + 1]; ++i) {
            c->part[i] = q;
            c->rho_n[i] = c->mat[c->pmat[q]].rho;
        }
    c->cw = (double *)malloc(sizeof(double) * M);
    c->s0 = (double *)malloc(sizeof(double) * M);
    c->Kn = (double *)malloc(sizeof(double) * M);
    c->E = (double *)malloc(sizeof(double) * M);
    for (int m = 0; m < M; ++m)
        material_constants(&c->mat[m], c->Rc, c->kn_mode, &c->cw[m], &c->s0[m], &c->Kn[m],
                           &c->E[m]);
    double **st[] = {&c->ux, &c->uy, &c->vx, &c->vy, &c->ax, &c->ay, &c->px, &c->py};
    for (int k = 0; k < 8; ++k) *st[k] = (double *)calloc((size_t)N > 0 ? N : 1, sizeof(double));
    for (int tt = 0; tt < NT; ++tt)
        for (int d = 0; d < 2; ++d)
            c->F[tt][d] = (double *)calloc((size_t)N > 0 ? N : 1, sizeof(double));
    if (p->u0x) memcpy(c->ux, p->u0x, sizeof(double) * N);
    if (p->u0y) memcpy(c->uy, p->u0y, sizeof(double) * N);
    if (p->v0x) memcpy(c->vx, p->v0x, sizeof(double) * N);
    if (p->v0y) memcpy(c->vy, p->v0y, sizeof(double) * N);
    int r = build_bonds(c);
    if (r != OR_OK) return r;
    setup_grid(c);
    /* t = 0: forces at u0, v0 with the break rule applied; a0 = F / (rho V) + g */
    c->step = 0;
    int s = eval_forces(c, c->vx, c->vy, 0.0);
    commit_breaks(c);
    accel_from_forces(c, c->ax, c->ay);
    c->status = s;
    return OR_OK;
}

void or_destroy(or_ctx *c) {
    if (!c) return;
    void *ptrs[] = {c->x, c->y, c->vol, c->rho_n, c->part, c->poff, c->pmat, c->pagg, c->mat,
                    c->cw, c->s0, c->Kn, c->E, c->loff, c->lvoff, c->lxy, c->box, c->vtop,
                    c->row, c->col, c->l0, c->broken, c->brk_eval, c->ux, c->uy, c->vx, c->vy,
                    c->ax, c->ay, c->px, c->py, c->agg_cell0, c->agg_ncx, c->agg_ncy,
                    c->agg_gx0, c->agg_gy0, c->cell_head, c->cell_next, c->node_cell};
    for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; ++k) free(ptrs[k]);
    for (int tt = 0; tt < NT; ++tt) {
        free(c->F[tt][0]);
        free(c->F[tt][1]);
    }
    free(c);
}

/* ------------------------------------------------------------------------ */
/* Algorithm alg:buildtree                                                   */
/* ------------------------------------------------------------------------ */
int or_step(or_ctx *c, int64_t n_steps) {
    if (c->status != OR_OK) return c->status;
    const int N = c->N;
    const double dt = c->dt, hdt2 = 0.5 * dt * dt, hdt = 0.5 * dt;
    double *anx = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *any = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    for (int64_t s = 0; s < n_steps; ++s) {
        /* u <- u + dt v + dt^2/2 a */
        for (int i = 0; i < N; ++i) {
            c->ux[i] = c->ux[i] + dt * c->vx[i] + hdt2 * c->ax[i];
            c->uy[i] = c->uy[i] + dt * c->vy[i] + hdt2 * c->ay[i];
        }
        c->step += 1;
        const double t = (double)c->step * dt;
        /* forces at the new positions with the old velocities */
        int st = eval_forces(c, c->vx, c->vy, t);
        commit_breaks(c);
        accel_from_forces(c, anx, any);
        /* v <- v + dt/2 (a_old + a_new) */
        for (int i = 0; i < N; ++i) {
            c->vx[i] = c->vx[i] + hdt * (c->ax[i] + anx[i]);
            c->vy[i] = c->vy[i] + hdt * (c->ay[i] + any[i]);
            c->ax[i] = anx[i];
            c->ay[i] = any[i];
        }
        if (st == OR_OK) st = check_finite(c);
        if (st != OR_OK) {
            c->status = st;
            break;
        }
    }
    free(anx);
    free(any);
    return c->status;
}

int or_forces(or_ctx *c, uint32_t mask, double *fx, double *fy) {
    const double t = (double)c->step * c->dt;
    int64_t saved[8];
    memcpy(saved, c->cnt, sizeof saved);
    eval_forces(c, c->vx, c->vy, t);
    memcpy(c->cnt, saved, sizeof saved); /* evaluation only: counters unchanged */
    for (int i = 0; i < c->N; ++i) {
        double sx = 0.0, sy = 0.0;
        for (int tt = 0; tt < NT; ++tt)
            if (mask & (1u << tt)) {
                sx += c->F[tt][0][i];
                sy += c->F[tt][1][i];
            }
        fx[i] = sx / c->vol[i];
        fy[i] = sy / c->vol[i];
    }
    return OR_OK;
}

/* Sec. 3.1: damage = broken bonds / reference bonds at the node */
/* Force the particles exert on each wall at the current state (positions
 * x + u, velocities v, top wall at time step * dt): minus the sum over the
 * aggregate's nodes of each wall's share of the wall force (Sec. 4.5, with a
 * corner correction split evenly between its two walls).
 * out[8 a + 2 w + k], walls w = left, right, floor, top; k = x, y. */
int or_wall_reactions(or_ctx *c, double *out) {
    const int N = c->N;
    for (int i = 0; i < N; ++i) {
        c->px[i] = c->x[i] + c->ux[i];
        c->py[i] = c->y[i] + c->uy[i];
    }
    for (int k = 0; k < 8 * c->A; ++k) out[k] = 0.0;
    const double t = (double)c->step * c->dt;
    int64_t cnt[8] = {0};
    int st = OR_OK;
    for (int i = 0; i < N; ++i) {
        double split[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const int s = wall_node_split(c, i, t, c->vx, c->vy, cnt, split);
        if (s != OR_OK) st = s;
        const int a = c->pagg[c->part[i]];
        for (int k = 0; k < 8; ++k) out[8 * a + k] -= split[k];
    }
    return st;
}

int or_damage(const or_ctx *c, double *phi, int64_t *nb) {
    int64_t tot = 0;
    for (int i = 0; i < c->N; ++i) {
        int nref = c->row[i + 1] - c->row[i], nbk = 0;
        for (int k = c->row[i]; k < c->row[i + 1]; ++k) nbk += c->broken[k];
        tot += nbk;
        if (phi) phi[i] = nref > 0 ? (double)nbk / (double)nref : 0.0;
    }
    if (nb) *nb = tot;
    return OR_OK;
}

int64_t or_contacts(or_ctx *c, int32_t *pi, int32_t *pj, int64_t cap) {
    for (int i = 0; i < c->N; ++i) {
        c->px[i] = c->x[i] + c->ux[i];
        c->py[i] = c->y[i] + c->uy[i];
    }
    int64_t n = 0;
    for (int i = 0; i < c->N; ++i)
        for (int j = i + 1; j < c->N; ++j) {
            if (c->pagg[c->part[j]] != c->pagg[c->part[i]]) continue;
            double dx = c->px[j] - c->px[i], dy = c->py[j] - c->py[i];
            double r2 = dx * dx + dy * dy;
            if (r2 < c->Rc2) {
                if (n < cap) {
                    pi[n] = i;
                    pj[n] = j;
                }
                ++n;
            }
        }
    return n;
}

int or_get_state(const or_ctx *c, double *ux, double *uy, double *vx, double *vy, double *ax,
                 double *ay, uint8_t *broken, int64_t *step) {
    size_t b = sizeof(double) * (size_t)c->N;
    if (ux) memcpy(ux, c->ux, b);
    if (uy) memcpy(uy, c->uy, b);
    if (vx) memcpy(vx, c->vx, b);
    if (vy) memcpy(vy, c->vy, b);
    if (ax) memcpy(ax, c->ax, b);
    if (ay) memcpy(ay, c->ay, b);
    if (broken) memcpy(broken, c->broken, (size_t)c->nnz);
    if (step) *step = c->step;
    return OR_OK;
}

int or_set_state(or_ctx *c, const double *ux, const double *uy, const double *vx,
                 const double *vy, const double *ax, const double *ay, const uint8_t *broken,
                 int64_t step) {
    size_t b = sizeof(double) * (size_t)c->N;
    memcpy(c->ux, ux, b);
    memcpy(c->uy, uy, b);
    memcpy(c->vx, vx, b);
    memcpy(c->vy, vy, b);
    memcpy(c->ax, ax, b);
    memcpy(c->ay, ay, b);
    if (broken) memcpy(c->broken, broken, (size_t)c->nnz);
    c->step = step;
    c->status = OR_OK;
    return OR_OK;
}

int or_counters(const or_ctx *c, int64_t out[8]) {
    memcpy(out, c->cnt, sizeof(int64_t) * 8);
    return OR_OK;
}
