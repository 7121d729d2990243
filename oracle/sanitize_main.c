/*
 * sanitize_main.c -- a driver that runs every entry point of the oracle on a
 * small problem, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (TEST INFRASTRUCTURE: built and run by the CPU tests only).
 *
 * The problem: a lattice disk, a plus-shaped particle (a non-convex boundary
 * loop, so that the line-of-sight filter of Sec. 5 runs) and a ring (a hole,
 * a clockwise loop), pushed together near the floor and a corner of the box
 * with a moving top wall, so that bonds break, self-contact and
 * inter-particle contact, walls and corners all act.  Exit status 0 when
 * every call succeeds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pd_oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define CHECK(x)                                                   \
    do {                                                           \
        if (!(x)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

static int inside_poly(const double *v, int n, double x, double y) {
    int in = 0;
    for (int i = 0, j = n - 1; i < n; j = i++) {
        const double xi = v[2 * i], yi = v[2 * i + 1], xj = v[2 * j], yj = v[2 * j + 1];
        if ((yi > y) != (yj > y) && x < xi + (y - yi) * (xj - xi) / (yj - yi)) in = !in;
    }
    return in;
}

int main(void) {
    const double h = 1e-4, R = 8 * h, Rc = 0.95 * h;
    /* plus: arm half-length R, half-width R/4 (12 vertices, counter-clockwise) */
    const double a = R, w = R / 4;
    const double plus[24] = {w, -a, w, -w, a, -w, a, w, w, w, w, a,
                             -w, a, -w, w, -a, w, -a, -w, -w, -w, -w, -a};
    enum { NC = 32 };
    double ring_out[2 * NC], ring_in[2 * NC];
    for (int k = 0; k < NC; ++k) {
        const double t = 2 * M_PI * k / NC;
        ring_out[2 * k] = R * cos(t);
        ring_out[2 * k + 1] = R * sin(t);
        ring_in[2 * k] = 0.5 * R * cos(-t);
        ring_in[2 * k + 1] = 0.5 * R * sin(-t);
    }
    const double cx[3] = {1.0e-3, 2.75e-3, 4.5e-3}, cy[3] = {0.85e-3, 0.9e-3, 0.95e-3};
    double *x = malloc(sizeof(double) * 4000), *y = malloc(sizeof(double) * 4000);
    int32_t po[4] = {0, 0, 0, 0};
    int n = 0;
    for (int p = 0; p < 3; ++p) {
        for (int j = -9; j <= 9; ++j)
            for (int i = -9; i <= 9; ++i) {
                const double bx = i * h, by = j * h;
                int keep;
                if (p == 0)
                    keep = bx * bx + by * by <= R * R;
                else if (p == 1)
                    keep = inside_poly(plus, 12, bx + 1e-3 * h, by + 2e-3 * h);
                else
                    keep = inside_poly(ring_out, NC, bx, by) && !inside_poly(ring_in, NC, bx, by);
                if (keep) {
                    x[n] = cx[p] + bx;
                    y[n] = cy[p] + by;
                    ++n;
                }
            }
        po[p + 1] = n;
    }
    double *vol = malloc(sizeof(double) * n), *vx = malloc(sizeof(double) * n),
           *vy = malloc(sizeof(double) * n);
    for (int k = 0; k < n; ++k) {
        vol[k] = h * h;
        vx[k] = (k < po[1]) ? 30.0 : ((k < po[2]) ? 0.0 : -30.0);
        vy[k] = -5.0;
    }
    const int32_t pm[3] = {0, 1, 0}, pa[3] = {0, 0, 0};
    const int32_t loff[4] = {0, 0, 1, 3};
    const int32_t lvoff[4] = {0, 12, 12 + NC, 12 + 2 * NC};
    double lxy[2 * (12 + 2 * NC)];
    for (int k = 0; k < 12; ++k) {
        lxy[2 * k] = cx[1] + plus[2 * k];
        lxy[2 * k + 1] = cy[1] + plus[2 * k + 1];
    }
    for (int k = 0; k < NC; ++k) {
        lxy[2 * (12 + k)] = cx[2] + ring_out[2 * k];
        lxy[2 * (12 + k) + 1] = cy[2] + ring_out[2 * k + 1];
        lxy[2 * (12 + NC + k)] = cx[2] + ring_in[2 * k];
        lxy[2 * (12 + NC + k) + 1] = cy[2] + ring_in[2 * k + 1];
    }
    const or_material mats[2] = {{1200.0, 2.16e7, 0.0, 5.0, 3 * h, 0},
                                 {2400.0, 6.0e7, 0.0, 8.0, 3.5 * h, 1}};
    const double box[4] = {0.0, 5.5e-3, 0.0, 2.0e-3};
    const double vtop[1] = {2.0};
    for (int mode = 0; mode < 2; ++mode) {
        or_problem pr;
        memset(&pr, 0, sizeof pr);
        pr.n_nodes = n;
        pr.n_particles = 3;
        pr.n_aggregates = 1;
        pr.n_materials = 2;
        pr.x = x;
        pr.y = y;
        pr.vol = vol;
        pr.particle_offset = po;
        pr.particle_material = pm;
        pr.particle_aggregate = pa;
        pr.materials = mats;
        pr.loop_offset = loff;
        pr.loop_vertex_offset = lvoff;
        pr.loop_xy = lxy;
        pr.v0x = vx;
        pr.v0y = vy;
        pr.contact_radius = Rc;
        pr.friction_mu = 0.5;
        pr.damping_ratio = 0.8;
        pr.kn_mode = mode;
        pr.box = box;
        pr.top_wall_speed = vtop;
        pr.gravity_y = -5000.0;
        pr.dt = mode ? 5e-9 : 2e-8;
        pr.contact_mode = mode;
        pr.n_threads = 1;
        or_ctx *c = NULL;
        CHECK(or_create(&pr, &c) == OR_OK);
        double k4[8];
        CHECK(or_constants(c, k4) == OR_OK);
        const int64_t nnz = or_n_bonds(c);
        CHECK(nnz > 0);
        int32_t *row = malloc(sizeof(int32_t) * (n + 1)), *col = malloc(sizeof(int32_t) * nnz);
        CHECK(or_bonds(c, row, col) == OR_OK);
        const int st = or_step(c, 300);
        CHECK(st == OR_OK || st == OR_E_ESCAPED);
        double *fx = malloc(sizeof(double) * n), *fy = malloc(sizeof(double) * n);
        const int sf = or_forces(c, 31, fx, fy);
        CHECK(sf == OR_OK || sf == OR_E_ESCAPED);
        double reac[8];
        or_wall_reactions(c, reac);
        double *phi = malloc(sizeof(double) * n);
        int64_t nb = 0;
        CHECK(or_damage(c, phi, &nb) == OR_OK);
        const int64_t ncont = or_contacts(c, NULL, NULL, 0);
        CHECK(ncont >= 0);
        int32_t *ci = malloc(sizeof(int32_t) * (ncont + 1)), *cj = malloc(sizeof(int32_t) * (ncont + 1));
        CHECK(or_contacts(c, ci, cj, ncont) == ncont);
        double *s[6];
        for (int k = 0; k < 6; ++k) s[k] = malloc(sizeof(double) * n);
        uint8_t *brk = malloc(nnz);
        int64_t step = 0;
        CHECK(or_get_state(c, s[0], s[1], s[2], s[3], s[4], s[5], brk, &step) == OR_OK);
        CHECK(or_set_state(c, s[0], s[1], s[2], s[3], s[4], s[5], brk, step) == OR_OK);
        int64_t cnt[8];
        CHECK(or_counters(c, cnt) == OR_OK);
        printf("mode %d: %d nodes, %lld bonds, %lld broken, %lld contacts, counters %lld %lld %lld %lld %lld\n",
               mode, n, (long long)nnz, (long long)nb, (long long)ncont, (long long)cnt[0],
               (long long)cnt[1], (long long)cnt[2], (long long)cnt[3], (long long)cnt[4]);
        CHECK(or_segment_in_particle(c, 1, cx[1], cy[1], cx[1] + 0.9 * a, cy[1]) == 1);
        CHECK(or_segment_in_particle(c, 1, cx[1] + 0.9 * a, cy[1] + 0.2 * w,
                                     cx[1] + 0.2 * w, cy[1] + 0.9 * a) == 0);
        for (int k = 0; k < 6; ++k) free(s[k]);
        free(brk);
        free(ci);
        free(cj);
        free(phi);
        free(fx);
        free(fy);
        free(row);
        free(col);
        or_destroy(c);
    }
    /* the wall regions over the whole range of signed distances */
    for (int i = -20; i <= 20; ++i) {
        double A, g, Ix, Iy;
        const double d = 0.999 * Rc * i / 20.0;
        or_wall_segment(Rc, d, &A, &g);
        CHECK(A >= 0.0 && isfinite(g));
        CHECK(isfinite(or_wall_segment_gap(Rc, d)));
        for (int j = -20; j <= 20; ++j) {
            or_wall_corner(Rc, d, 0.999 * Rc * j / 20.0, &A, &Ix, &Iy);
            CHECK(isfinite(A) && isfinite(Ix) && isfinite(Iy));
        }
    }
    free(x);
    free(y);
    free(vol);
    free(vx);
    free(vy);
    printf("ok\n");
    return 0;
}
