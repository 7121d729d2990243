// pd_host.cpp -- host side of libpd: setup, step orchestration, C ABI.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "pd_internal.h"

using namespace pd;

struct pd_ctx {
    Ctx c;
};

namespace {

constexpr double kPi = 3.14159265358979323846;

pd_status fail(Ctx &c, pd_status st, const std::string &m) {
    c.err = m;
    return st;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(c, PD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

template <typename T>
pd_status dalloc(Ctx &c, T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return fail(c, PD_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c.owned.push_back(q);
    *p = (T *)q;
    return PD_OK;
}

template <typename T>
pd_status upload(Ctx &c, T **p, const T *src, size_t n) {
    pd_status s = dalloc(c, p, n);
    if (s != PD_OK) return s;
    if (n) {
        hipError_t e = hipMemcpyAsync(*p, src, n * sizeof(T), hipMemcpyHostToDevice, c.stream);
        if (e != hipSuccess) return fail(c, PD_E_DEVICE, hipGetErrorString(e));
    }
    return PD_OK;
}

#define TRY(expr)                          \
    do {                                   \
        pd_status s_ = (expr);             \
        if (s_ != PD_OK) return s_;        \
    } while (0)

// per-material constants: Table tab:2d-peri (c_w, s0), nu = 1/3 in 2-D, K_n
MatConst material_constants(const pd_material &m, double Rc, int kn_mode) {
    MatConst k{};
    const double nu = 1.0 / 3.0;
    const double eps = m.horizon;
    const double E = m.young_E > 0.0 ? m.young_E : 2.0 * m.bulk_k * (1.0 - nu);
    const double e3 = eps * eps * eps;
    if (m.micro == PD_MICRO_CONST) {
        k.cw = 6.0 * E / (kPi * e3 * (1.0 - nu));
        k.s0 = sqrt(4.0 * kPi * m.Gc / (9.0 * E * eps));
        k.conic = 0;
    } else {
        k.cw = 24.0 * E / (kPi * e3 * (1.0 - nu));
        k.s0 = sqrt(5.0 * kPi * m.Gc / (9.0 * E * eps));
        k.conic = 1;
    }
    k.Kn = kn_mode == PD_KN_SELF_CONSISTENT ? k.cw / Rc
                                             : 18.0 * m.bulk_k / (kPi * e3 * eps * eps);
    k.eps = eps;
    k.rho = m.rho;
    k.Kd_self = k.cw / Rc;
    return k;
}

// Barrier segments of one particle (Sec. 5): every boundary edge moved out by
// delta along the exterior-angle bisectors of its end vertices, plus, at each
// non-convex vertex, the bisector ray up to its first hit with the boundary
// (or to the bounding circle when it hits nothing).  A candidate bond that
// properly crosses one of them leaves the particle.
void barrier_segments(const double *xy, const int *vert_off, int l0, int l1, double cx, double cy,
                      double rmax, double delta, std::vector<double> &out) {
    struct E {
        double ax, ay, bx, by;
    };
    std::vector<E> edges;
    for (int l = l0; l < l1; ++l) {
        const int v0 = vert_off[l], n = vert_off[l + 1] - v0;
        for (int k = 0; k < n; ++k) {
            const int k1 = (k + 1) % n;
            edges.push_back({xy[2 * (v0 + k)], xy[2 * (v0 + k) + 1], xy[2 * (v0 + k1)],
                             xy[2 * (v0 + k1) + 1]});
        }
    }
    for (int l = l0; l < l1; ++l) {
        const int v0 = vert_off[l], n = vert_off[l + 1] - v0;
        if (n < 3) continue;
        std::vector<double> ex(n), ey(n);  // pushed vertices
        for (int k = 0; k < n; ++k) {
            const int km = (k + n - 1) % n, kp = (k + 1) % n;
            const double px = xy[2 * (v0 + k)], py = xy[2 * (v0 + k) + 1];
            double ax = px - xy[2 * (v0 + km)], ay = py - xy[2 * (v0 + km) + 1];
            double bx = xy[2 * (v0 + kp)] - px, by = xy[2 * (v0 + kp) + 1] - py;
            const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
            ax /= la;
            ay /= la;
            bx /= lb;
            by /= lb;
            const double cr = ax * by - ay * bx;  // v_{i-1} x v_i
            double nx, ny;
            if (cr != 0.0) {
                // unit bisector of the exterior angle
                nx = bx - ax;
                ny = by - ay;
                const double ln = sqrt(nx * nx + ny * ny);
                nx /= ln;
                ny /= ln;
                if (cr > 0.0) {  // convex vertex: flip to point outward
                    nx = -nx;
                    ny = -ny;
                }
            } else {  // straight: outward normal of a loop with the domain on its left
                nx = by;
                ny = -bx;
            }
            ex[k] = px + delta * nx;
            ey[k] = py + delta * ny;
            if (cr < 0.0) {  // non-convex cusp: bisector ray to the first boundary hit
                double tbest = sqrt((px - cx) * (px - cx) + (py - cy) * (py - cy)) + rmax;
                for (const E &e : edges) {
                    const bool incident = (e.ax == px && e.ay == py) || (e.bx == px && e.by == py);
                    if (incident) continue;
                    const double sx = e.bx - e.ax, sy = e.by - e.ay;
                    const double den = nx * sy - ny * sx;
                    if (den == 0.0) continue;
                    const double wx = e.ax - px, wy = e.ay - py;
                    const double t = (wx * sy - wy * sx) / den;
                    const double u = (wx * ny - wy * nx) / den;
                    if (t > 0.0 && u >= 0.0 && u <= 1.0 && t < tbest) tbest = t;
                }
                // start a hair outside the vertex: a bond through the vertex itself
                // touches the closed domain and is kept
                const double tau = 1e-9 * delta;  // 1e-12 of the horizon
                out.insert(out.end(), {px + tau * nx, py + tau * ny, px + tbest * nx, py + tbest * ny});
            }
        }
        for (int k = 0; k < n; ++k) {
            const int kp = (k + 1) % n;
            out.insert(out.end(), {ex[k], ey[k], ex[kp], ey[kp]});
        }
    }
}

void set_state_ptrs(Ctx &c, int cur) {
    DevArgs &a = c.a;
    const int nx = cur ^ 1;
    a.ux = c.U[cur][0];
    a.uy = c.U[cur][1];
    a.vx = c.V[cur][0];
    a.vy = c.V[cur][1];
    a.ax = c.Acc[cur][0];
    a.ay = c.Acc[cur][1];
    a.ux_o = c.U[nx][0];
    a.uy_o = c.U[nx][1];
    a.vx_o = c.V[nx][0];
    a.vy_o = c.V[nx][1];
    a.ax_o = c.Acc[nx][0];
    a.ay_o = c.Acc[nx][1];
}

int lds_cap(const Ctx &c) { return c.tune.use_lds ? force_lds_cap(c.max_win) : 0; }

// radix sort of c.a.keys into skey/perm
hipError_t enqueue_sort(Ctx &c, hipEvent_t *ev) {
    const int P = c.a.radix_passes;
    const uint32_t *kin = c.a.keys;
    const int *vin = nullptr;
    for (int p = 0; p < P; ++p) {
        const bool last_parity = ((P - 1 - p) % 2) == 0;
        uint32_t *kout = last_parity ? c.skey_buf : c.keys_alt;
        int *vout = last_parity ? c.perm_buf : c.perm_alt;
        hipError_t e = launch_sort_pass(kin, vin, kout, vout, c.N, kRadixBits * p, c.hist, c.dtotal,
                                        c.stream, ev ? ev + 4 * p : nullptr);
        if (e != hipSuccess) return e;
        kin = kout;
        vin = vout;
    }
    return hipSuccess;
}

// positions -> keys -> sort -> cells, at the current (adv = 0) or advanced
// (adv = 1) positions of buffer cur
hipError_t enqueue_search(Ctx &c, int cur, int adv, int advance_step) {
    set_state_ptrs(c, cur);
    hipError_t e = launch_keys(c.a, adv, c.stream);
    if (e != hipSuccess) return e;
    e = enqueue_sort(c, nullptr);
    if (e != hipSuccess) return e;
    return launch_cells(c.a, adv, advance_step, c.stream);
}

hipError_t enqueue_step(Ctx &c, int cur) {
    hipError_t e = enqueue_search(c, cur, 1, 1);
    if (e != hipSuccess) return e;
    set_state_ptrs(c, cur);
    return launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream);
}

pd_status build_windows(Ctx &c) {
    const int B = c.tune.block_nodes;
    const int nb = (c.N + B - 1) / B;
    if (c.win_lo) {
        hipFree(c.win_lo);
        hipFree(c.win_hi);
        c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), (void *)c.win_lo), c.owned.end());
        c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), (void *)c.win_hi), c.owned.end());
    }
    TRY(dalloc(c, &c.win_lo, nb));
    TRY(dalloc(c, &c.win_hi, nb));
    HIPCHK(launch_fill_u32((uint32_t *)c.win_lo, 0x7fffffffu, nb, c.stream));
    HIPCHK(launch_fill_u32((uint32_t *)c.win_hi, 0u, nb, c.stream));
    c.a.block_nodes = B;
    c.a.win_lo = c.win_lo;
    c.a.win_hi = c.win_hi;
    HIPCHK(launch_windows(c.a, c.win_lo, c.win_hi, c.stream));
    std::vector<int> lo(nb), hi(nb);
    HIPCHK(hipMemcpyAsync(lo.data(), c.win_lo, nb * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(hi.data(), c.win_hi, nb * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    int mw = 0;
    for (int b = 0; b < nb; ++b) mw = std::max(mw, hi[b] - lo[b] + 1);
    c.max_win = mw;
    return PD_OK;
}

double list_radius(const Ctx &c) { return c.a.Rc * (1.0 + c.tune.skin_factor); }

void set_list_params(Ctx &c) {
    const double r = list_radius(c);
    c.a.Rl2 = r * r;
    const double m = 0.45 * c.tune.skin_factor * c.a.Rc;  // half the skin, with a margin
    c.a.move2 = m * m;
}

pd_status build_grid(Ctx &c, const double *box) {
    const double cs = c.tune.cell_factor * list_radius(c);
    c.h_gx0.assign(c.A, 0);
    c.h_gy0.assign(c.A, 0);
    c.h_ncx.assign(c.A, 0);
    c.h_ncy.assign(c.A, 0);
    c.h_cell0.assign(c.A, 0);
    uint64_t nc = 0;
    for (int a = 0; a < c.A; ++a) {
        const double xlo = box[4 * a], xhi = box[4 * a + 1], ylo = box[4 * a + 2], yhi = box[4 * a + 3];
        c.h_gx0[a] = xlo - 2.0 * cs;
        c.h_gy0[a] = ylo - 2.0 * cs;
        c.h_ncx[a] = (int)((xhi - xlo) / cs) + 5;
        c.h_ncy[a] = (int)((yhi - ylo) / cs) + 5;
        c.h_cell0[a] = (uint32_t)nc;
        nc += (uint64_t)c.h_ncx[a] * (uint64_t)c.h_ncy[a];
        if (nc >= 0xffffffffull) return fail(c, PD_E_INVALID, "too many cells: raise cell_factor");
    }
    c.ncells = (int64_t)nc;
    int bits = 1;
    while (bits < 32 && (1ull << bits) < nc) ++bits;
    c.a.radix_passes = (bits + kRadixBits - 1) / kRadixBits;
    double *gx0, *gy0;
    int *ncx, *ncy;
    uint32_t *cell0, *cs_buf;
    TRY(upload(c, &gx0, c.h_gx0.data(), c.A));
    TRY(upload(c, &gy0, c.h_gy0.data(), c.A));
    TRY(upload(c, &ncx, c.h_ncx.data(), c.A));
    TRY(upload(c, &ncy, c.h_ncy.data(), c.A));
    TRY(upload(c, &cell0, c.h_cell0.data(), c.A));
    TRY(dalloc(c, &cs_buf, (size_t)nc));
    HIPCHK(launch_fill_u32(cs_buf, 0u, (int64_t)nc, c.stream));
    c.a.agg_gx0 = gx0;
    c.a.agg_gy0 = gy0;
    c.a.agg_ncx = ncx;
    c.a.agg_ncy = ncy;
    c.a.agg_cell0 = cell0;
    c.a.cell_start = cs_buf;
    c.a.cell = cs;
    c.a.inv_cell = 1.0 / cs;
    return PD_OK;
}

void invalidate_graph(Ctx &c) {
    for (int k = 0; k < 2; ++k) {
        if (c.graph[k]) {
            hipGraphExecDestroy(c.graph[k]);
            c.graph[k] = nullptr;
        }
        if (c.lgraph[k]) {
            hipGraphExecDestroy(c.lgraph[k]);
            c.lgraph[k] = nullptr;
        }
    }
    c.graph_valid = false;
}

// list-mode replay: kChunk steps from buffer parity `start`
hipError_t enqueue_list_steps(Ctx &c, int start, int n) {
    for (int k = 0; k < n; ++k) {
        set_state_ptrs(c, (start + k) & 1);
        c.a.chunk_k = k;
        hipError_t e = launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, true);
        if (e != hipSuccess) return e;
    }
    c.a.chunk_k = 0;
    return hipSuccess;
}

pd_status ensure_list_graph(Ctx &c) {
    if (c.lgraph[0] && c.lgraph[1]) return PD_OK;
    for (int start = 0; start < 2; ++start) {
        if (c.lgraph[start]) continue;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
        hipError_t e1 = enqueue_list_steps(c, start, kChunk);
        hipError_t e2 = hipStreamEndCapture(c.stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return fail(c, PD_E_DEVICE, "graph capture failed");
        }
        hipError_t e3 = hipGraphInstantiate(&c.lgraph[start], g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(c, PD_E_DEVICE, "graph instantiate failed");
    }
    return PD_OK;
}

pd_status ensure_graph(Ctx &c) {
    if (c.graph_valid) return PD_OK;
    invalidate_graph(c);
    for (int start = 0; start < 2; ++start) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
        hipError_t e1 = enqueue_step(c, start);
        hipError_t e2 = enqueue_step(c, start ^ 1);
        hipError_t e3 = hipStreamEndCapture(c.stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return fail(c, PD_E_DEVICE, "graph capture failed");
        }
        hipError_t e4 = hipGraphInstantiate(&c.graph[start], g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e4 != hipSuccess) return fail(c, PD_E_DEVICE, "graph instantiate failed");
    }
    c.graph_valid = true;
    return PD_OK;
}

pd_status read_status(Ctx &c) {
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, c.a.status, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (st & kStNonfinite) c.status = PD_E_NONFINITE;
    else if (st & kStEscaped) c.status = PD_E_ESCAPED;
    if (c.status) return fail(c, (pd_status)c.status,
                              c.status == PD_E_NONFINITE ? "non-finite state" : "node escaped a wall");
    return PD_OK;
}

pd_status set_device_step(Ctx &c) {
    HIPCHK(launch_set_u64((unsigned long long *)c.a.step, (unsigned long long)c.step, c.stream));
    return PD_OK;
}

// forces at the current state into the term buffer (M_FORCES)
pd_status eval_terms(Ctx &c) {
    if (!c.a.terms) TRY(dalloc(c, &c.a.terms, (size_t)10 * c.N));
    HIPCHK(enqueue_search(c, c.cur, 0, 0));
    set_state_ptrs(c, c.cur);
    HIPCHK(launch_force(c.a, c.precision, M_FORCES, lds_cap(c), c.stream));
    return PD_OK;
}

pd_status alloc_lists(Ctx &c, int maxc) {
    if (c.a.clist) {
        hipFree(c.a.clist);
        c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), (void *)c.a.clist), c.owned.end());
        c.a.clist = nullptr;
    }
    TRY(dalloc(c, &c.a.clist, (size_t)maxc * c.N));
    c.a.maxc = maxc;
    invalidate_graph(c);
    return PD_OK;
}

// candidate lists at the advanced positions of the current state: keys, radix
// sort and cell starts there, then the per-node lists
pd_status rebuild_lists(Ctx &c, hipEvent_t *ev = nullptr, float *ms = nullptr) {
    for (int attempt = 0; attempt < 4; ++attempt) {
        HIPCHK(hipMemsetAsync(c.a.overflow, 0, sizeof(int), c.stream));
        set_state_ptrs(c, c.cur);
        if (ev) HIPCHK(hipEventRecord(ev[0], c.stream));
        HIPCHK(launch_keys(c.a, 1, c.stream));
        if (ev) HIPCHK(hipEventRecord(ev[1], c.stream));
        HIPCHK(enqueue_sort(c, ev ? ev + 2 : nullptr));
        const int b = 2 + 4 * c.a.radix_passes;
        if (ev) HIPCHK(hipEventRecord(ev[b], c.stream));
        HIPCHK(launch_cells(c.a, 1, 0, c.stream));
        if (ev) HIPCHK(hipEventRecord(ev[b + 1], c.stream));
        HIPCHK(launch_build_list(c.a, c.stream));
        if (ev) HIPCHK(hipEventRecord(ev[b + 2], c.stream));
        HIPCHK(launch_invalidate(c.a, ~0ull, c.stream));
        int over = 0;
        HIPCHK(hipMemcpyAsync(&over, c.a.overflow, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        if (over == 0) {
            c.list_valid = true;
            ++c.rebuilds;
            return PD_OK;
        }
        int m = c.a.maxc;
        while (m < over) m *= 2;
        TRY(alloc_lists(c, m));
    }
    return fail(c, PD_E_DEVICE, "candidate lists keep overflowing");
}

// list-mode steps: replays of up to kChunk steps; a replay stops early when a
// list goes stale (a node moved half the skin, or a bond broke), then the
// lists are rebuilt and the remaining steps run
pd_status step_lists(Ctx &c, int64_t n) {
    int64_t left = n;
    while (left > 0) {
        if (!c.list_valid) TRY(rebuild_lists(c));
        HIPCHK(launch_invalidate(c.a, ~0ull, c.stream));
        HIPCHK(launch_set_u64((unsigned long long *)c.a.step_base, (unsigned long long)c.step,
                              c.stream));
        const int chunk = (int)std::min<int64_t>(left, kChunk);
        if (c.tune.use_graph && chunk == kChunk) {
            TRY(ensure_list_graph(c));
            HIPCHK(hipGraphLaunch(c.lgraph[c.cur], c.stream));
        } else {
            HIPCHK(enqueue_list_steps(c, c.cur, chunk));
        }
        unsigned long long inv = 0;
        int st = 0;
        HIPCHK(hipMemcpyAsync(&inv, c.a.invalid_step, sizeof(inv), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipMemcpyAsync(&st, c.a.status, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        int64_t done = chunk;
        if (inv != ~0ull) {
            const int64_t lim = (int64_t)inv - 1 - c.step;  // steps that ran
            done = std::max<int64_t>(0, std::min<int64_t>(chunk, lim));
        }
        c.cur = (int)((c.cur + done) & 1);
        c.step += done;
        left -= done;
        if (inv != ~0ull && (int64_t)inv <= c.step + 1) c.list_valid = false;
        if (st) return read_status(c);
    }
    set_state_ptrs(c, c.cur);
    TRY(set_device_step(c));
    return PD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *pd_last_error(const pd_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->c.err.c_str();
}

void pd_destroy(pd_ctx *ctx) {
    if (!ctx) return;
    Ctx &c = ctx->c;
    if (c.stream) hipStreamSynchronize(c.stream);
    invalidate_graph(c);
    for (void *p : c.owned) hipFree(p);
    if (c.own_stream && c.stream) hipStreamDestroy(c.stream);
    delete ctx;
}

pd_status pd_setup(const pd_problem *p, pd_ctx **out) {
    if (!out) return PD_E_INVALID;
    *out = nullptr;
    pd_ctx *ctx = new (std::nothrow) pd_ctx();
    if (!ctx) return PD_E_NOMEM;
    *out = ctx;
    Ctx &c = ctx->c;
    if (!p) return fail(c, PD_E_INVALID, "null problem");
    // ---- validation ----
    const int N = p->n_nodes, P = p->n_particles, M = p->n_materials;
    const int A = p->n_aggregates > 0 ? p->n_aggregates : 1;
    if (N < 1 || P < 1 || M < 1) return fail(c, PD_E_INVALID, "empty problem");
    if (!p->x || !p->y || !p->vol || !p->particle_offset || !p->particle_material ||
        !p->materials || !p->box)
        return fail(c, PD_E_INVALID, "missing array");
    if (!(p->dt > 0.0) || !(p->contact_radius > 0.0))
        return fail(c, PD_E_INVALID, "dt and contact_radius must be positive");
    if (p->precision != PD_PREC_FP64 && p->precision != PD_PREC_FP32_FORCE)
        return fail(c, PD_E_INVALID, "bad precision");
    if (p->particle_offset[0] != 0 || p->particle_offset[P] != N)
        return fail(c, PD_E_INVALID, "particle offsets must start at 0 and end at n_nodes");
    for (int q = 0; q < P; ++q) {
        if (p->particle_offset[q + 1] <= p->particle_offset[q])
            return fail(c, PD_E_INVALID, "empty particle or unordered offsets");
        if (p->particle_material[q] < 0 || p->particle_material[q] >= M)
            return fail(c, PD_E_INVALID, "bad material index");
        if (p->particle_aggregate && (p->particle_aggregate[q] < 0 || p->particle_aggregate[q] >= A))
            return fail(c, PD_E_INVALID, "bad aggregate index");
    }
    for (int m = 0; m < M; ++m)
        if (!(p->materials[m].horizon > 0.0) || !(p->materials[m].rho > 0.0))
            return fail(c, PD_E_INVALID, "material horizon and density must be positive");
    for (int i = 0; i < N; ++i)
        if (!(p->vol[i] > 0.0)) return fail(c, PD_E_INVALID, "nodal volume must be positive");
    if (p->loop_offset) {
        const int nl = p->loop_offset[P];
        if (p->loop_offset[0] != 0 || nl < 0 || (nl > 0 && (!p->loop_vertex_offset || !p->loop_xy)))
            return fail(c, PD_E_INVALID, "bad loop offsets");
        for (int l = 0; l < nl; ++l)
            if (p->loop_vertex_offset[l + 1] - p->loop_vertex_offset[l] < 3)
                return fail(c, PD_E_INVALID, "a boundary loop needs at least 3 vertices");
    }
    c.N = N;
    c.P = P;
    c.A = A;
    c.M = M;
    c.precision = p->precision;
    // ---- stream ----
    if (p->hip_stream) {
        c.stream = (hipStream_t)p->hip_stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        c.own_stream = true;
    }
    // ---- host-side per node / particle data ----
    std::vector<int> part(N), pagg(P, 0);
    for (int q = 0; q < P; ++q) {
        for (int i = p->particle_offset[q]; i < p->particle_offset[q + 1]; ++i) part[i] = q;
        if (p->particle_aggregate) pagg[q] = p->particle_aggregate[q];
    }
    std::vector<MatConst> mc(M);
    for (int m = 0; m < M; ++m) mc[m] = material_constants(p->materials[m], p->contact_radius, p->kn_mode);
    std::vector<double> mass(N);
    for (int i = 0; i < N; ++i) mass[i] = p->materials[p->particle_material[part[i]]].rho * p->vol[i];
    // initial positions inside the boxes
    for (int i = 0; i < N; ++i) {
        const int a = pagg[part[i]];
        const double px = p->x[i] + (p->u0x ? p->u0x[i] : 0.0);
        const double py = p->y[i] + (p->u0y ? p->u0y[i] : 0.0);
        const double *b = p->box + 4 * a;
        if (!(px - b[0] > -p->contact_radius && b[1] - px > -p->contact_radius &&
              py - b[2] > -p->contact_radius && b[3] - py > -p->contact_radius))
            return fail(c, PD_E_INVALID, "node outside its box");
    }
    // ---- scalars ----
    DevArgs &a = c.a;
    a.N = N;
    a.P = P;
    a.A = A;
    a.M = M;
    a.Rc = p->contact_radius;
    a.Rc2 = p->contact_radius * p->contact_radius;
    a.mu = p->friction_mu;
    a.rd = p->damping_ratio;
    a.dt = p->dt;
    a.hdt = 0.5 * p->dt;
    a.hdt2 = 0.5 * p->dt * p->dt;
    a.gx = p->gravity_x;
    a.gy = p->gravity_y;
    // ---- device copies ----
    double *dx, *dy, *dvol, *dmass, *dbox, *dvtop;
    int *dpart, *dpmat, *dpagg, *dpoff;
    MatConst *dmat;
    TRY(upload(c, &dx, p->x, N));
    TRY(upload(c, &dy, p->y, N));
    TRY(upload(c, &dvol, p->vol, N));
    TRY(upload(c, &dmass, mass.data(), N));
    TRY(upload(c, &dpart, part.data(), N));
    TRY(upload(c, &dpmat, p->particle_material, P));
    TRY(upload(c, &dpagg, pagg.data(), P));
    TRY(upload(c, &dpoff, p->particle_offset, P + 1));
    TRY(upload(c, &dmat, mc.data(), M));
    TRY(upload(c, &dbox, p->box, 4 * (size_t)A));
    std::vector<double> vtop(A, 0.0);
    if (p->top_wall_speed)
        for (int q = 0; q < A; ++q) vtop[q] = p->top_wall_speed[q];
    TRY(upload(c, &dvtop, vtop.data(), A));
    a.x = dx;
    a.y = dy;
    a.vol = dvol;
    a.mass = dmass;
    a.part = dpart;
    a.pmat = dpmat;
    a.pagg = dpagg;
    a.mat = dmat;
    a.box = dbox;
    a.vtop = dvtop;
    // state buffers
    std::vector<double> zero(N, 0.0);
    for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d) {
            TRY(dalloc(c, &c.U[b][d], N));
            TRY(dalloc(c, &c.V[b][d], N));
            TRY(dalloc(c, &c.Acc[b][d], N));
        }
    const double *init[4] = {p->u0x, p->u0y, p->v0x, p->v0y};
    double *dst[4] = {c.U[0][0], c.U[0][1], c.V[0][0], c.V[0][1]};
    for (int k = 0; k < 4; ++k)
        HIPCHK(hipMemcpyAsync(dst[k], init[k] ? init[k] : zero.data(), N * sizeof(double),
                              hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(c.Acc[0][0], zero.data(), N * sizeof(double), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(c.Acc[0][1], zero.data(), N * sizeof(double), hipMemcpyHostToDevice, c.stream));
    c.cur = 0;
    // ---- reference bonds ----
    std::vector<double> seg;
    std::vector<int> seg_off(P + 1, 0);
    for (int q = 0; q < P; ++q) {
        seg_off[q] = (int)(seg.size() / 4);
        if (p->loop_offset && p->loop_offset[q + 1] > p->loop_offset[q]) {
            double cx = 0, cy = 0;
            const int i0 = p->particle_offset[q], i1 = p->particle_offset[q + 1];
            for (int i = i0; i < i1; ++i) {
                cx += p->x[i];
                cy += p->y[i];
            }
            cx /= (i1 - i0);
            cy /= (i1 - i0);
            double rmax = 0;
            for (int l = p->loop_offset[q]; l < p->loop_offset[q + 1]; ++l)
                for (int v = p->loop_vertex_offset[l]; v < p->loop_vertex_offset[l + 1]; ++v)
                    rmax = std::max(rmax, hypot(p->loop_xy[2 * v] - cx, p->loop_xy[2 * v + 1] - cy));
            const double delta = 1e-3 * p->materials[p->particle_material[q]].horizon;
            const size_t s_begin = seg.size();
            barrier_segments(p->loop_xy, p->loop_vertex_offset, p->loop_offset[q],
                             p->loop_offset[q + 1], cx, cy, rmax, delta, seg);
            // particle frame: relative to the particle's first node
            const double rx = p->x[i0], ry = p->y[i0];
            for (size_t k = s_begin; k < seg.size(); k += 2) {
                seg[k] -= rx;
                seg[k + 1] -= ry;
            }
        }
    }
    seg_off[P] = (int)(seg.size() / 4);
    std::vector<double> thr2(M);
    for (int m = 0; m < M; ++m) {
        const double e = p->materials[m].horizon;
        const double t = e - 1e-9 * e;
        thr2[m] = t * t;
    }
    double *dseg, *dthr2;
    int *dsegoff, *drowlen;
    TRY(upload(c, &dseg, seg.data(), seg.size()));
    TRY(upload(c, &dsegoff, seg_off.data(), P + 1));
    TRY(upload(c, &dthr2, thr2.data(), M));
    TRY(dalloc(c, &drowlen, N));
    BondArgs ba{dx, dy, dpart, dpmat, dpoff, dseg, dsegoff, dthr2, N};
    HIPCHK(launch_bonds_count(ba, drowlen, c.stream));
    c.h_rowlen.resize(N);
    HIPCHK(hipMemcpyAsync(c.h_rowlen.data(), drowlen, N * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const int S = (N + kSlice - 1) / kSlice;
    c.h_slice_ptr.assign(S + 1, 0);
    int64_t nnz = 0, slots = 0;
    for (int s = 0; s < S; ++s) {
        int w = 0;
        for (int i = s * kSlice; i < std::min(N, (s + 1) * kSlice); ++i) {
            w = std::max(w, c.h_rowlen[i]);
            nnz += c.h_rowlen[i];
        }
        slots += (int64_t)w * kSlice;
        if (slots >= 0xffffffffll) return fail(c, PD_E_INVALID, "too many bonds");
        c.h_slice_ptr[s + 1] = (uint32_t)slots;
    }
    c.nnz = nnz;
    c.nslots = slots;
    uint32_t *dsp, *dcol;
    TRY(upload(c, &dsp, c.h_slice_ptr.data(), S + 1));
    TRY(dalloc(c, &dcol, (size_t)slots));
    HIPCHK(launch_fill_u32(dcol, kBroken, slots, c.stream));
    HIPCHK(launch_bonds_fill(ba, dcol, dsp, c.stream));
    a.col = dcol;
    a.slice_ptr = dsp;
    a.rowlen = drowlen;
    a.n_slices = S;
    // ---- contact search buffers ----
    set_list_params(c);
    TRY(build_grid(c, p->box));
    TRY(dalloc(c, &a.keys, N));
    TRY(dalloc(c, &c.keys_alt, N));
    TRY(dalloc(c, &c.skey_buf, N));
    TRY(dalloc(c, &c.perm_buf, N));
    TRY(dalloc(c, &c.perm_alt, N));
    const int G = (N + kSortTile - 1) / kSortTile;
    TRY(dalloc(c, &c.hist, (size_t)kRadix * G));
    TRY(dalloc(c, &c.dtotal, kRadix));
    a.skey = c.skey_buf;
    a.perm = c.perm_buf;
    TRY(dalloc(c, &a.spx, N));
    TRY(dalloc(c, &a.spy, N));
    TRY(dalloc(c, &a.spart, N));
    TRY(dalloc(c, &a.step, 1));
    TRY(dalloc(c, &a.step_base, 1));
    TRY(dalloc(c, &a.invalid_step, 1));
    TRY(dalloc(c, &a.overflow, 1));
    TRY(dalloc(c, &a.clist_n, N));
    TRY(dalloc(c, &a.ubx, N));
    TRY(dalloc(c, &a.uby, N));
    TRY(alloc_lists(c, 16));
    HIPCHK(launch_invalidate(a, ~0ull, c.stream));
    TRY(dalloc(c, &a.status, 1));
    TRY(dalloc(c, &a.counters, C_N));
    HIPCHK(hipMemsetAsync(a.status, 0, sizeof(int), c.stream));
    HIPCHK(hipMemsetAsync(a.counters, 0, sizeof(unsigned long long) * C_N, c.stream));
    c.step = 0;
    TRY(set_device_step(c));
    a.use_lds = c.tune.use_lds;
    TRY(build_windows(c));
    // ---- t = 0: forces at u0, v0 with the break rule; a0 = F / (rho V) + g ----
    HIPCHK(enqueue_search(c, 0, 0, 0));
    set_state_ptrs(c, 0);
    a.ax_o = c.Acc[0][0];
    a.ay_o = c.Acc[0][1];
    HIPCHK(launch_force(a, c.precision, M_PROLOGUE, lds_cap(c), c.stream));
    set_state_ptrs(c, 0);
    HIPCHK(hipStreamSynchronize(c.stream));
    pd_status st = read_status(c);
    if (st != PD_OK) {
        // the state at t = 0 is already outside the admissible set; keep it sticky
        return PD_OK;
    }
    return PD_OK;
}

pd_status pd_step(pd_ctx *ctx, int64_t n) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (n < 0) return fail(c, PD_E_INVALID, "negative step count");
    if (c.status) return (pd_status)c.status;
    if (n == 0) return PD_OK;
    if (c.tune.skin_factor > 0.0) {
        TRY(step_lists(c, n));
        return read_status(c);
    }
    int64_t left = n;
    if (c.tune.use_graph) {
        TRY(ensure_graph(c));
        while (left >= 2) {
            HIPCHK(hipGraphLaunch(c.graph[c.cur], c.stream));
            left -= 2;  // two steps bring the buffers back to the same parity
        }
    }
    while (left > 0) {
        HIPCHK(enqueue_step(c, c.cur));
        c.cur ^= 1;
        --left;
    }
    set_state_ptrs(c, c.cur);
    c.step += n;
    pd_status st = read_status(c);
    return st;
}

pd_status pd_forces(pd_ctx *ctx, uint32_t mask, double *fx, double *fy, int32_t on_device) {
    if (!ctx || !fx || !fy) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(eval_terms(c));
    double *ox = fx, *oy = fy;
    if (!on_device) {
        if (!c.dev_d) TRY(dalloc(c, &c.dev_d, 2 * (size_t)c.N));
        ox = c.dev_d;
        oy = c.dev_d + c.N;
    }
    HIPCHK(launch_sum_terms(c.a, mask, ox, oy, c.stream));
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(fx, ox, c.N * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipMemcpyAsync(fy, oy, c.N * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_damage(pd_ctx *ctx, double *phi, int64_t *nb, int32_t on_device) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    unsigned long long *dnb;
    if (!c.dev_i) TRY(dalloc(c, &c.dev_i, 4));
    dnb = (unsigned long long *)c.dev_i;
    HIPCHK(hipMemsetAsync(dnb, 0, sizeof(unsigned long long), c.stream));
    double *dphi = nullptr;
    if (phi) {
        if (on_device) {
            dphi = phi;
        } else {
            if (!c.dev_d) TRY(dalloc(c, &c.dev_d, 2 * (size_t)c.N));
            dphi = c.dev_d;
        }
    }
    HIPCHK(launch_damage(c.a, dphi, dnb, c.stream));
    unsigned long long h = 0;
    HIPCHK(hipMemcpyAsync(&h, dnb, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    if (phi && !on_device)
        HIPCHK(hipMemcpyAsync(phi, dphi, c.N * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (nb) *nb = (int64_t)h;
    return PD_OK;
}

int64_t pd_n_bonds(const pd_ctx *ctx) { return ctx ? ctx->c.nnz : -1; }

static pd_status download_col(Ctx &c, std::vector<uint32_t> &col) {
    col.resize((size_t)c.nslots);
    HIPCHK(hipMemcpyAsync(col.data(), c.a.col, c.nslots * sizeof(uint32_t), hipMemcpyDeviceToHost,
                          c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_bonds(pd_ctx *ctx, int32_t *row, int32_t *col) {
    if (!ctx || !row || !col) return PD_E_INVALID;
    Ctx &c = ctx->c;
    std::vector<uint32_t> h;
    TRY(download_col(c, h));
    int64_t w = 0;
    for (int i = 0; i < c.N; ++i) {
        row[i] = (int32_t)w;
        const uint32_t base = c.h_slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
        for (int k = 0; k < c.h_rowlen[i]; ++k) col[w++] = (int32_t)(h[base + (uint32_t)k * kSlice] & kIndexMask);
    }
    row[c.N] = (int32_t)w;
    return PD_OK;
}

pd_status pd_contacts(pd_ctx *ctx, int32_t *pi, int32_t *pj, int64_t cap, int64_t *count) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    HIPCHK(enqueue_search(c, c.cur, 0, 0));
    set_state_ptrs(c, c.cur);
    int *dcnt;
    long long *doff;
    TRY(dalloc(c, &dcnt, c.N));
    TRY(dalloc(c, &doff, c.N + 1));
    HIPCHK(launch_contacts_count(c.a, dcnt, c.stream));
    std::vector<int> cnt(c.N);
    HIPCHK(hipMemcpyAsync(cnt.data(), dcnt, c.N * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    std::vector<long long> off(c.N + 1, 0);
    for (int i = 0; i < c.N; ++i) off[i + 1] = off[i] + cnt[i];
    const long long tot = off[c.N];
    if (count) *count = tot;
    std::vector<int> hi((size_t)std::max<long long>(tot, 1)), hj((size_t)std::max<long long>(tot, 1));
    if (tot > 0) {
        int *dpi, *dpj;
        TRY(dalloc(c, &dpi, (size_t)tot));
        TRY(dalloc(c, &dpj, (size_t)tot));
        HIPCHK(hipMemcpyAsync(doff, off.data(), (c.N + 1) * sizeof(long long), hipMemcpyHostToDevice, c.stream));
        HIPCHK(launch_contacts_fill(c.a, doff, dpi, dpj, c.stream));
        HIPCHK(hipMemcpyAsync(hi.data(), dpi, tot * sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipMemcpyAsync(hj.data(), dpj, tot * sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        for (void *q : {(void *)dpi, (void *)dpj}) {
            hipFree(q);
            c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), q), c.owned.end());
        }
    }
    for (void *q : {(void *)dcnt, (void *)doff}) {
        hipFree(q);
        c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), q), c.owned.end());
    }
    std::vector<std::pair<int, int>> pr((size_t)tot);
    for (long long k = 0; k < tot; ++k) pr[k] = {hi[k], hj[k]};
    std::sort(pr.begin(), pr.end());
    for (long long k = 0; k < std::min<long long>(tot, cap); ++k) {
        pi[k] = pr[k].first;
        pj[k] = pr[k].second;
    }
    return PD_OK;
}

pd_status pd_get_state(pd_ctx *ctx, double *ux, double *uy, double *vx, double *vy, double *ax,
                       double *ay, uint8_t *broken, int64_t *step) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    double *dst[6] = {ux, uy, vx, vy, ax, ay};
    const double *src[6] = {c.U[c.cur][0], c.U[c.cur][1], c.V[c.cur][0], c.V[c.cur][1],
                            c.Acc[c.cur][0], c.Acc[c.cur][1]};
    for (int k = 0; k < 6; ++k)
        if (dst[k])
            HIPCHK(hipMemcpyAsync(dst[k], src[k], c.N * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (broken) {
        std::vector<uint32_t> h;
        TRY(download_col(c, h));
        int64_t w = 0;
        for (int i = 0; i < c.N; ++i) {
            const uint32_t base = c.h_slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
            for (int k = 0; k < c.h_rowlen[i]; ++k) broken[w++] = (h[base + (uint32_t)k * kSlice] & kBroken) ? 1 : 0;
        }
    }
    if (step) *step = c.step;
    return PD_OK;
}

pd_status pd_set_state(pd_ctx *ctx, const double *ux, const double *uy, const double *vx,
                       const double *vy, const double *ax, const double *ay,
                       const uint8_t *broken, int64_t step) {
    if (!ctx || !ux || !uy || !vx || !vy || !ax || !ay) return PD_E_INVALID;
    Ctx &c = ctx->c;
    HIPCHK(hipStreamSynchronize(c.stream));
    c.cur = 0;
    const double *src[6] = {ux, uy, vx, vy, ax, ay};
    double *dst[6] = {c.U[0][0], c.U[0][1], c.V[0][0], c.V[0][1], c.Acc[0][0], c.Acc[0][1]};
    for (int k = 0; k < 6; ++k)
        HIPCHK(hipMemcpyAsync(dst[k], src[k], c.N * sizeof(double), hipMemcpyHostToDevice, c.stream));
    if (broken) {
        std::vector<uint32_t> h;
        TRY(download_col(c, h));
        int64_t w = 0;
        for (int i = 0; i < c.N; ++i) {
            const uint32_t base = c.h_slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
            for (int k = 0; k < c.h_rowlen[i]; ++k) {
                uint32_t &e = h[base + (uint32_t)k * kSlice];
                e = broken[w++] ? (e | kBroken) : (e & kIndexMask);
            }
        }
        HIPCHK(hipMemcpyAsync(c.a.col, h.data(), c.nslots * sizeof(uint32_t), hipMemcpyHostToDevice,
                              c.stream));
    }
    c.step = step;
    TRY(set_device_step(c));
    HIPCHK(hipMemsetAsync(c.a.status, 0, sizeof(int), c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    c.status = 0;
    c.list_valid = false;
    set_state_ptrs(c, 0);
    return PD_OK;
}

pd_status pd_counters(pd_ctx *ctx, int64_t out[8]) {
    if (!ctx || !out) return PD_E_INVALID;
    Ctx &c = ctx->c;
    unsigned long long h[C_N];
    HIPCHK(hipMemcpyAsync(h, c.a.counters, sizeof h, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    for (int k = 0; k < 7; ++k) out[k] = (int64_t)h[k];
    out[7] = c.step;
    return PD_OK;
}

pd_status pd_set_counting(pd_ctx *ctx, int32_t on) {
    if (!ctx) return PD_E_INVALID;
    ctx->c.a.counting = on ? 1 : 0;
    invalidate_graph(ctx->c);
    return PD_OK;
}

pd_status pd_get_tuning(const pd_ctx *ctx, pd_tuning *t) {
    if (!ctx || !t) return PD_E_INVALID;
    *t = ctx->c.tune;
    return PD_OK;
}

pd_status pd_set_tuning(pd_ctx *ctx, const pd_tuning *t) {
    if (!ctx || !t) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!(t->block_nodes == 64 || t->block_nodes == 128 || t->block_nodes == 256))
        return fail(c, PD_E_INVALID, "block_nodes must be 64, 128 or 256");
    if (!(t->cell_factor >= 1.0) || t->cell_factor > 64.0)
        return fail(c, PD_E_INVALID, "cell_factor must be in [1, 64]");
    if (!(t->skin_factor >= 0.0) || t->skin_factor > 16.0)
        return fail(c, PD_E_INVALID, "skin_factor must be in [0, 16]");
    HIPCHK(hipStreamSynchronize(c.stream));
    const bool regrid = t->cell_factor != c.tune.cell_factor || t->skin_factor != c.tune.skin_factor;
    const bool rewin = t->block_nodes != c.tune.block_nodes;
    c.tune = *t;
    c.tune.use_lds = t->use_lds ? 1 : 0;
    c.tune.use_graph = t->use_graph ? 1 : 0;
    c.a.use_lds = c.tune.use_lds;
    c.list_valid = false;
    set_list_params(c);
    if (regrid) {
        std::vector<double> box(4 * (size_t)c.A);
        HIPCHK(hipMemcpy(box.data(), c.a.box, box.size() * sizeof(double), hipMemcpyDeviceToHost));
        // release the old grid arrays
        const void *old[] = {c.a.agg_gx0, c.a.agg_gy0, c.a.agg_ncx, c.a.agg_ncy, c.a.agg_cell0,
                             c.a.cell_start};
        for (const void *q : old) {
            hipFree((void *)q);
            c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), q), c.owned.end());
        }
        TRY(build_grid(c, box.data()));
    }
    if (rewin) TRY(build_windows(c));
    invalidate_graph(c);
    return PD_OK;
}

pd_status pd_sizes(const pd_ctx *ctx, int64_t out[10]) {
    if (!ctx || !out) return PD_E_INVALID;
    const Ctx &c = ctx->c;
    out[0] = c.N;
    out[1] = c.nnz;
    out[2] = c.nslots;
    out[3] = c.ncells;
    out[4] = c.a.radix_passes;
    out[5] = c.P;
    out[6] = c.A;
    out[7] = c.max_win;
    out[8] = c.rebuilds;
    out[9] = c.a.maxc;
    return PD_OK;
}

pd_status pd_time_kernels(pd_ctx *ctx, int64_t n_steps, double *ms, int32_t *launches, int32_t n_out) {
    if (!ctx || !ms || n_out < 7 || n_steps < 1) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (c.status) return (pd_status)c.status;
    const int P = c.a.radix_passes;
    const int nev = 2 + 4 * P + 3;
    std::vector<hipEvent_t> ev(nev), fe(2);
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    for (auto &e : fe) HIPCHK(hipEventCreate(&e));
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    int32_t cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    const bool list = c.tune.skin_factor > 0.0;
    auto add_search = [&](bool with_list) -> pd_status {
        float t;
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        acc[0] += t;
        cnt[0] += 1;
        for (int p = 0; p < P; ++p) {
            hipEvent_t *e = ev.data() + 2 + 4 * p;
            HIPCHK(hipEventElapsedTime(&t, e[0], e[1]));
            acc[1] += t;
            HIPCHK(hipEventElapsedTime(&t, e[1], e[2]));
            acc[2] += t;
            HIPCHK(hipEventElapsedTime(&t, e[2], e[3]));
            acc[3] += t;
            cnt[1] += 1;
            cnt[2] += 1;
            cnt[3] += 1;
        }
        const int b = 2 + 4 * P;
        HIPCHK(hipEventElapsedTime(&t, ev[b], ev[b + 1]));
        acc[4] += t;
        cnt[4] += 1;
        if (with_list) {
            HIPCHK(hipEventElapsedTime(&t, ev[b + 1], ev[b + 2]));
            acc[6] += t;
            cnt[6] += 1;
        }
        return PD_OK;
    };
    int64_t s = 0;
    while (s < n_steps) {
        if (list) {
            if (!c.list_valid) {
                TRY(rebuild_lists(c, ev.data()));
                TRY(add_search(true));
            }
            // a run of back-to-back step launches between two events
            const int run = (int)std::min<int64_t>(n_steps - s, kChunk);
            HIPCHK(launch_invalidate(c.a, ~0ull, c.stream));
            HIPCHK(launch_set_u64((unsigned long long *)c.a.step_base, (unsigned long long)c.step,
                                  c.stream));
            HIPCHK(hipEventRecord(fe[0], c.stream));
            HIPCHK(enqueue_list_steps(c, c.cur, run));
            HIPCHK(hipEventRecord(fe[1], c.stream));
            unsigned long long inv = 0;
            HIPCHK(hipMemcpyAsync(&inv, c.a.invalid_step, sizeof(inv), hipMemcpyDeviceToHost, c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));
            int64_t done = run;
            if (inv != ~0ull) done = std::max<int64_t>(0, std::min<int64_t>(run, (int64_t)inv - 1 - c.step));
            if (done == run) {  // only complete runs time the kernel
                float t;
                HIPCHK(hipEventElapsedTime(&t, fe[0], fe[1]));
                acc[5] += t;
                cnt[5] += run;
            }
            c.cur = (int)((c.cur + done) & 1);
            c.step += done;
            s += std::max<int64_t>(done, 1);
            if (inv != ~0ull && (int64_t)inv <= c.step + 1) c.list_valid = false;
        } else {
            set_state_ptrs(c, c.cur);
            HIPCHK(hipEventRecord(ev[0], c.stream));
            HIPCHK(launch_keys(c.a, 1, c.stream));
            HIPCHK(hipEventRecord(ev[1], c.stream));
            HIPCHK(enqueue_sort(c, ev.data() + 2));
            const int b = 2 + 4 * P;
            HIPCHK(hipEventRecord(ev[b], c.stream));
            HIPCHK(launch_cells(c.a, 1, 1, c.stream));
            HIPCHK(hipEventRecord(ev[b + 1], c.stream));
            set_state_ptrs(c, c.cur);
            HIPCHK(hipEventRecord(fe[0], c.stream));
            HIPCHK(launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, false));
            HIPCHK(hipEventRecord(fe[1], c.stream));
            HIPCHK(hipEventSynchronize(fe[1]));
            TRY(add_search(false));
            float t;
            HIPCHK(hipEventElapsedTime(&t, fe[0], fe[1]));
            acc[5] += t;
            cnt[5] += 1;
            c.cur ^= 1;
            c.step += 1;
            ++s;
        }
    }
    set_state_ptrs(c, c.cur);
    if (list) TRY(set_device_step(c));
    for (auto &e : ev) hipEventDestroy(e);
    for (auto &e : fe) hipEventDestroy(e);
    for (int k = 0; k < 7; ++k) {
        ms[k] = cnt[k] ? acc[k] / (double)cnt[k] : 0.0;
        if (launches) launches[k] = cnt[k];
    }
    return read_status(c);
}

pd_status pd_autotune(pd_ctx *ctx, int32_t steps, pd_tuning *chosen) {
    if (!ctx || steps < 1) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (c.status) return (pd_status)c.status;
    // save the state (device-side copies)
    const size_t nb = c.N * sizeof(double);
    double *save;
    uint32_t *save_col;
    TRY(dalloc(c, &save, 6 * (size_t)c.N));
    TRY(dalloc(c, &save_col, (size_t)c.nslots));
    const int cur0 = c.cur;
    const long long step0 = c.step;
    double *src[6] = {c.U[cur0][0], c.U[cur0][1], c.V[cur0][0], c.V[cur0][1], c.Acc[cur0][0], c.Acc[cur0][1]};
    for (int k = 0; k < 6; ++k)
        HIPCHK(hipMemcpyAsync(save + k * c.N, src[k], nb, hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(save_col, c.a.col, c.nslots * sizeof(uint32_t), hipMemcpyDeviceToDevice, c.stream));
    unsigned long long cnt_save[C_N];
    HIPCHK(hipMemcpyAsync(cnt_save, c.a.counters, sizeof cnt_save, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const pd_tuning base = c.tune;
    pd_tuning best = base;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int blocks[3] = {256, 128, 64};
    const double skins[4] = {0.0, 0.5, 1.0, 2.0};
    pd_status result = PD_OK;
    for (int bi = 0; bi < 3 && result == PD_OK; ++bi)
        for (int ci = 0; ci < 4 && result == PD_OK; ++ci)
            for (int li = 0; li < 2 && result == PD_OK; ++li) {
                pd_tuning t = base;
                t.block_nodes = blocks[bi];
                t.cell_factor = 1.0;
                t.skin_factor = skins[ci];
                t.use_lds = 1 - li;
                if ((result = pd_set_tuning(ctx, &t)) != PD_OK) break;
                // restore and warm up
                for (int k = 0; k < 6; ++k)
                    HIPCHK(hipMemcpyAsync(src[k], save + k * c.N, nb, hipMemcpyDeviceToDevice, c.stream));
                c.cur = cur0;
                c.step = step0;
                TRY(set_device_step(c));
                if ((result = pd_step(ctx, 2)) != PD_OK) break;
                HIPCHK(hipEventRecord(e0, c.stream));
                if ((result = pd_step(ctx, steps)) != PD_OK) break;
                HIPCHK(hipEventRecord(e1, c.stream));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    pd_status s2 = pd_set_tuning(ctx, &best);
    for (int k = 0; k < 6; ++k)
        HIPCHK(hipMemcpyAsync(src[k], save + k * c.N, nb, hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(c.a.col, save_col, c.nslots * sizeof(uint32_t), hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(c.a.counters, cnt_save, sizeof cnt_save, hipMemcpyHostToDevice, c.stream));
    c.cur = cur0;
    c.step = step0;
    c.status = 0;
    HIPCHK(hipMemsetAsync(c.a.status, 0, sizeof(int), c.stream));
    TRY(set_device_step(c));
    HIPCHK(hipStreamSynchronize(c.stream));
    set_state_ptrs(c, c.cur);
    for (void *q : {(void *)save, (void *)save_col}) {
        hipFree(q);
        c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), q), c.owned.end());
    }
    if (chosen) *chosen = best;
    if (result != PD_OK) return result;
    return s2;
}

}  // extern "C"
