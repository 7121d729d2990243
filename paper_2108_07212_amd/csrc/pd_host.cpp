// pd_host.cpp -- host side of libpd: setup, step orchestration, C ABI.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "pd_internal.h"

using namespace pd;

struct pd_ctx {
    Ctx c;
};

// Workspace of pd_forces_noalloc: the per-term force densities of one
// evaluation, 10 doubles per node.  Every device the library runs on holds
// its own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol: its device address, per device, comes from
// hipGetSymbolAddress at pd_setup and is the only handle host code uses.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (the device must be current)
hipError_t scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
    return hipSuccess;
}

double *scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}
}  // namespace

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
    const double t = eps - 1e-9 * eps;  // as the bond build's threshold
    k.thr2 = t * t;
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
                    // a ray that meets the boundary at a vertex stops there: in a
                    // regular polygon of an even vertex count (a ring's hole) each
                    // cusp's ray runs through the opposite vertex, where rounding
                    // can leave u just outside both adjacent edges, and the ray
                    // would run on through the material behind
                    constexpr double kEnd = 1e-9;
                    if (t > 0.0 && u >= -kEnd && u <= 1.0 + kEnd && t < tbest) tbest = t;
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
    a.unx = c.UN[cur][0];
    a.uny = c.UN[cur][1];
    a.unx_o = c.UN[nx][0];
    a.uny_o = c.UN[nx][1];
}

int lds_cap(const Ctx &c) { return c.tune.use_lds ? force_lds_cap(c.max_win) : 0; }

// radix sort of c.a.keys into skey/perm (hist_done: the first pass's digit
// counts are already in c.hist)
hipError_t enqueue_sort(Ctx &c, hipEvent_t *ev, bool hist_done) {
    const int P = c.a.radix_passes;
    const uint32_t *kin = c.a.keys;
    const int *vin = nullptr;
    for (int p = 0; p < P; ++p) {
        const bool last_parity = ((P - 1 - p) % 2) == 0;
        uint32_t *kout = last_parity ? c.skey_buf : c.keys_alt;
        int *vout = last_parity ? c.perm_buf : c.perm_alt;
        hipError_t e = launch_sort_pass(kin, vin, kout, vout, c.N, kRadixBits * p, c.hist, c.dtotal,
                                        c.stream, ev ? ev + 4 * p : nullptr, hist_done && p == 0);
        if (e != hipSuccess) return e;
        kin = kout;
        vin = vout;
    }
    return hipSuccess;
}

// cell keys and their radix sort; ev: null, or the keys' two events then the
// sort's four per pass.  With one key per thread the keys kernel also counts
// the first pass's digits (its workgroups are that pass's tiles).
hipError_t enqueue_keys_sort(Ctx &c, int adv, hipEvent_t *ev) {
    const bool fuse = c.a.radix_passes > 0 && sort_items(c.N) == 1;
    hipError_t e = ev ? hipEventRecord(ev[0], c.stream) : hipSuccess;
    if (e != hipSuccess) return e;
    e = launch_keys(c.a, adv, fuse ? c.hist : nullptr, sort_tiles(c.N), c.stream);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], c.stream)) != hipSuccess) return e;
    return enqueue_sort(c, ev ? ev + 2 : nullptr, fuse);
}

// positions -> keys -> sort -> cells, at the current (adv = 0) or advanced
// (adv = 1) positions of buffer cur
hipError_t enqueue_search(Ctx &c, int cur, int adv, int advance_step) {
    set_state_ptrs(c, cur);
    hipError_t e = enqueue_keys_sort(c, adv, nullptr);
    if (e != hipSuccess) return e;
    return launch_cells(c.a, adv, advance_step, c.stream);
}

hipError_t enqueue_step(Ctx &c, int cur) {
    hipError_t e = enqueue_search(c, cur, 1, 1);
    if (e != hipSuccess) return e;
    set_state_ptrs(c, cur);
    // (the modal closure runs only with candidate lists: enqueue_list_steps)
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
    uint32_t *cell0, *cs_buf, *ce_buf;
    TRY(upload(c, &gx0, c.h_gx0.data(), c.A));
    TRY(upload(c, &gy0, c.h_gy0.data(), c.A));
    TRY(upload(c, &ncx, c.h_ncx.data(), c.A));
    TRY(upload(c, &ncy, c.h_ncy.data(), c.A));
    TRY(upload(c, &cell0, c.h_cell0.data(), c.A));
    TRY(dalloc(c, &cs_buf, (size_t)nc));
    TRY(dalloc(c, &ce_buf, (size_t)nc));
    HIPCHK(launch_fill_u32(cs_buf, 0u, (int64_t)nc, c.stream));
    HIPCHK(launch_fill_u32(ce_buf, 0u, (int64_t)nc, c.stream));
    c.a.agg_gx0 = gx0;
    c.a.agg_gy0 = gy0;
    c.a.agg_ncx = ncx;
    c.a.agg_ncy = ncy;
    c.a.agg_cell0 = cell0;
    c.a.cell_start = cs_buf;
    c.a.cell_end = ce_buf;
    c.a.cell = cs;
    c.a.inv_cell = 1.0 / cs;
    return PD_OK;
}

void invalidate_graph(Ctx &c) {
    for (auto &kv : c.lgraph_n) hipGraphExecDestroy(kv.second);
    c.lgraph_n.clear();
    for (int k = 0; k < 2; ++k) {
        if (c.graph[k]) {
            hipGraphExecDestroy(c.graph[k]);
            c.graph[k] = nullptr;
        }
        for (int w = 0; w < 2; ++w)
            if (c.lgraph[w][k]) {
                hipGraphExecDestroy(c.lgraph[w][k]);
                c.lgraph[w][k] = nullptr;
            }
    }
    c.graph_valid = false;
}

// the closure's kernels after the force kernel of one step: projection of
// the closure particles, the MLP (learned closure), nodal accelerations
hipError_t enqueue_closure(Ctx &c, bool list) {
    if (c.cl.mode == 0) return hipSuccess;
    if (c.cl.reduced) {
        // reduced state: one launch (contact of the active nodes, advance
        // and reduction, the MLP of the learned closure, the update)
        return launch_rc_fused(c.a, c.cl.ca, c.cl.ma, c.precision, c.cl.mode == 2, list, c.stream);
    }
    hipError_t e = launch_cl_project(c.a, c.cl.ca, list, 0, c.cl.max_n, c.stream);
    if (e != hipSuccess) return e;
    if (c.cl.mode == 2) {
        e = launch_mlp_forward(c.cl.ma, c.a, list, c.stream);
        if (e != hipSuccess) return e;
    }
    return launch_cl_apply(c.a, c.cl.ca, list, c.stream);
}

// list-mode replay: n steps from buffer parity `start`
// the pass of walls and contact candidates runs with candidate lists and the
// closure off
bool wall_pass_on(const Ctx &c) {
    return c.tune.wall_pass && c.tune.skin_factor > 0.0 && !c.cl.mode && c.a.wfx;
}

hipError_t enqueue_list_launches(Ctx &c, int start, int n) {
    for (int k = 0; k < n; ++k) {
        set_state_ptrs(c, (start + k) & 1);
        c.a.chunk_k = k;
        hipError_t e;
        if (c.cl.mode) {
            // plain-force particles, then the closure particles' contact and walls
            e = c.cl.plain_launch ? launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, true, 1)
                                  : hipSuccess;
            // (the reduced form evaluates its contact inside its step kernel)
            if (e == hipSuccess && !c.cl.reduced) e = launch_cl_contact(c.a, c.precision, c.stream);
        } else if (wall_pass_on(c)) {
            e = launch_pass(c.a, c.precision, c.stream);
            if (e == hipSuccess)
                e = launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, true, 0, true);
        } else {
            e = launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, true);
        }
        if (e != hipSuccess) return e;
        e = enqueue_closure(c, true);
        if (e != hipSuccess) return e;
    }
    c.a.chunk_k = 0;
    return hipSuccess;
}

hipError_t enqueue_list_steps(Ctx &c, int start, int n) {
    // (the closure kernels take their arguments by value at enqueue)
    c.cl.ca.stop_on_fallback = (c.cl.mode && !c.cl.plain_launch) ? 1 : 0;
    hipError_t e = enqueue_list_launches(c, start, n);
    c.cl.ca.stop_on_fallback = 0;
    c.a.chunk_k = 0;
    return e;
}

pd_status capture_list_graph(Ctx &c, int start, int n, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
    hipError_t e1 = enqueue_list_steps(c, start, n);
    hipError_t e2 = hipStreamEndCapture(c.stream, &g);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail(c, PD_E_DEVICE, "graph capture failed");
    }
    hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e3 != hipSuccess) return fail(c, PD_E_DEVICE, "graph instantiate failed");
    return PD_OK;
}

pd_status ensure_list_graph(Ctx &c) {
    hipGraphExec_t *g = c.lgraph[c.cl.plain_launch ? 1 : 0];
    for (int start = 0; start < 2; ++start)
        if (!g[start]) TRY(capture_list_graph(c, start, kChunk, &g[start]));
    return PD_OK;
}

// a replay of n < kChunk steps (short pd_step calls, the rest of a call, the
// steps up to a periodic closure check), captured once per length and parity
pd_status list_graph_n(Ctx &c, int start, int n, hipGraphExec_t *out) {
    const long key = ((long)(c.cl.plain_launch ? 1 : 0) * 2 + start) * 1000000L + n;
    auto it = c.lgraph_n.find(key);
    if (it == c.lgraph_n.end()) {
        hipGraphExec_t g = nullptr;
        TRY(capture_list_graph(c, start, n, &g));
        it = c.lgraph_n.emplace(key, g).first;
    }
    *out = it->second;
    return PD_OK;
}

hipError_t enqueue_rebuild(Ctx &c, hipEvent_t *ev);

// plain list mode: a rebuild of the lists, the replay's arming (no steps run
// if a list did not fit its slots) and n steps from buffer parity `start`
// (the current one), captured once per length and parity
pd_status rebuild_graph_n(Ctx &c, int start, int n, hipGraphExec_t *out) {
    const long key = (4L + start) * 1000000L + n;
    auto it = c.lgraph_n.find(key);
    if (it == c.lgraph_n.end()) {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
        hipError_t e1 = enqueue_rebuild(c, nullptr);
        if (e1 == hipSuccess) e1 = launch_arm_replay(c.a, c.stream);
        if (e1 == hipSuccess) e1 = enqueue_list_steps(c, start, n);
        hipError_t e2 = hipStreamEndCapture(c.stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return fail(c, PD_E_DEVICE, "graph capture failed");
        }
        hipGraphExec_t x = nullptr;
        hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(c, PD_E_DEVICE, "graph instantiate failed");
        it = c.lgraph_n.emplace(key, x).first;
    }
    *out = it->second;
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

// Work on device buffers the caller produced must follow the caller's work.
// Without a stream from the caller, the library runs on a stream of its own
// (the legacy default stream cannot be captured into graphs) that waits here
// for everything issued so far on the legacy default stream.
pd_status after_caller(Ctx &c) {
    if (!c.own_stream) return PD_OK;
    HIPCHK(hipEventRecord(c.caller_ev, nullptr));
    HIPCHK(hipStreamWaitEvent(c.stream, c.caller_ev, 0));
    return PD_OK;
}

pd_status rc_sync(Ctx &c);

// forces at the current state into the term buffer (M_FORCES)
pd_status eval_terms(Ctx &c) {
    TRY(rc_sync(c));
    if (!c.a.terms) TRY(dalloc(c, &c.a.terms, (size_t)10 * c.N));
    HIPCHK(enqueue_search(c, c.cur, 0, 0));
    set_state_ptrs(c, c.cur);
    HIPCHK(launch_force(c.a, c.precision, M_FORCES, lds_cap(c), c.stream));
    return PD_OK;
}

pd_status alloc_lists(Ctx &c, int maxc) {
    if (maxc > kBlMaxc)
        return fail(c, PD_E_DEVICE, "a node has more than " + std::to_string(kBlMaxc) +
                                        " contact candidates");
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

// reduced closure: every node of every active reduced particle written into
// the current nodal state (a step writes only the boundary nodes)
pd_status rc_sync(Ctx &c) {
    if (!(c.cl.ready && c.cl.mode && c.cl.reduced)) return PD_OK;
    set_state_ptrs(c, c.cur);
    HIPCHK(launch_rc_sync(c.a, c.cl.ca, c.stream));
    return PD_OK;
}

pd_status cl_block_list(Ctx &c);

// after a rebuild: the active nodes of every reduced particle (nodes with
// candidates, candidates, nodes near a wall), the motion bound's origin
pd_status rc_activate(Ctx &c) {
    ClState &L = c.cl;
    if (!(L.ready && L.mode && L.reduced)) return PD_OK;
    set_state_ptrs(c, c.cur);
    HIPCHK(hipMemsetAsync(L.act, 0, (size_t)c.N, c.stream));
    HIPCHK(launch_rc_mark(c.a, L.act, (double)(c.step + 1) * c.a.dt, c.stream));
    HIPCHK(launch_rc_collect(c.a, L.ca, L.act, c.stream));
    L.rb_step = c.step;
    return PD_OK;
}

// candidate lists at the advanced positions of the current state: keys, radix
// sort and cell starts there, then the per-node lists (enqueued only, after
// a round start with its rebuild flag, which clears the counters they fill;
// no memset, so that replays can capture it)
hipError_t enqueue_rebuild(Ctx &c, hipEvent_t *ev) {
    set_state_ptrs(c, c.cur);
    hipError_t e = enqueue_keys_sort(c, 1, ev);
    if (e != hipSuccess) return e;
    const int b = 2 + 4 * c.a.radix_passes;
    if (ev && (e = hipEventRecord(ev[b], c.stream)) != hipSuccess) return e;
    if ((e = launch_cells(c.a, 1, 0, c.stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[b + 1], c.stream)) != hipSuccess) return e;
    if ((e = launch_build_list(c.a, c.stream)) != hipSuccess) return e;
    if (wall_pass_on(c) && (e = launch_pass_mark(c.a, c.stream)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[b + 2], c.stream)) != hipSuccess) return e;
    return hipSuccess;
}

// a rebuild at the current step whose lists fit their slots
pd_status rebuild_done(Ctx &c) {
    c.list_valid = true;
    const double gap = (double)(c.step - c.last_rebuild_step);
    if (c.rebuilds > 0 && gap > 0.0)
        c.rebuild_interval = c.rebuild_interval > 1e8 ? gap : 0.5 * (c.rebuild_interval + gap);
    c.last_rebuild_step = c.step;
    ++c.rebuilds;
    return rc_activate(c);
}

// lists too short for a node's candidates: twice as many slots, until they fit
pd_status grow_lists(Ctx &c, int over) {
    int m = c.a.maxc;
    while (m < over) m *= 2;
    return alloc_lists(c, m);
}

// the lists rebuilt and checked before returning
pd_status rebuild_lists(Ctx &c, hipEvent_t *ev = nullptr, float *ms = nullptr) {
    TRY(rc_sync(c));
    for (int attempt = 0; attempt < 4; ++attempt) {
        HIPCHK(launch_round_start(c.a, c.step, true, c.stream));
        HIPCHK(enqueue_rebuild(c, ev));
        HIPCHK(launch_invalidate(c.a, ~0ull, c.stream));
        int over = 0;
        HIPCHK(hipMemcpyAsync(&over, c.a.overflow, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        if (over == 0) return rebuild_done(c);
        TRY(grow_lists(c, over));
    }
    return fail(c, PD_E_DEVICE, "candidate lists keep overflowing");
}

// list-mode steps: replays of up to kChunk steps; a replay stops early when a
// list goes stale (a node moved half the skin, or a bond broke), then the
// lists are rebuilt and the remaining steps run
pd_status closure_check(Ctx &c);

pd_status step_lists(Ctx &c, int64_t n) {
    int64_t left = n;
    while (left > 0) {
        // the closure's periodic check against the plain bond force
        if (c.cl.mode && c.cl.check_every > 0 && c.step % c.cl.check_every == 0 &&
            c.step != c.cl.last_check_step) {
            TRY(closure_check(c));
            c.cl.last_check_step = c.step;
        }
        // reduced closure and the pass: the moving top wall may approach a
        // node that is not listed (active, near a wall) by at most half the
        // skin between rebuilds
        int64_t n_wall = 0;
        const int64_t rb_step = (c.cl.mode && c.cl.reduced) ? c.cl.rb_step : c.last_rebuild_step;
        if ((c.cl.mode && c.cl.reduced) || wall_pass_on(c)) {
            double vmax = 0.0;
            for (double v : c.h_vtop) vmax = std::max(vmax, fabs(v));
            const double skin = sqrt(c.a.Rl2) - c.a.Rc;
            if (vmax > 0.0) n_wall = std::max<int64_t>(1, (int64_t)floor(0.5 * skin / (vmax * c.a.dt)));
            if (n_wall > 0 && c.step - rb_step >= n_wall) c.list_valid = false;
        }
        // plain steps queue the rebuild ahead of the replay (one graph), whose
        // steps run only if every list fit its slots (checked with the
        // replay's results)
        bool queued_rebuild = false;
        if (!c.list_valid) {
            if (c.cl.mode)
                TRY(rebuild_lists(c));
            else
                queued_rebuild = true;
        }
        // closure on: the plain-force launch only while some particle is under
        // the plain force (a particle leaving the closure ends a replay without it)
        c.cl.plain_launch = true;
        if (c.cl.mode) {
            HIPCHK(hipMemcpyAsync(&c.rb->npb, c.cl.n_pd_blocks, sizeof(int), hipMemcpyDeviceToHost,
                                  c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));
            c.cl.plain_launch = c.rb->npb > 0;
        }
        HIPCHK(launch_round_start(c.a, c.step, queued_rebuild, c.stream));
        int64_t lim = std::min<int64_t>(left, kChunk);
        // lists that go stale within a replay: replays of about 1.5 times the
        // usual interval (a multiple of 8 steps), so that few launches run as
        // no-ops after a stale step
        if (c.rebuild_interval < kChunk) {
            const int64_t len = 8 * (int64_t)ceil(1.5 * c.rebuild_interval / 8.0);
            lim = std::min<int64_t>(lim, std::max<int64_t>(8, len));
        }
        if (c.cl.mode && c.cl.check_every > 0)
            lim = std::min<int64_t>(lim, c.cl.check_every - c.step % c.cl.check_every);
        if (n_wall > 0) {
            // (a rebuild queued ahead of this replay is at the current step)
            const int64_t rbs = queued_rebuild                   ? c.step
                                : (c.cl.mode && c.cl.reduced) ? c.cl.rb_step
                                                              : c.last_rebuild_step;
            lim = std::min<int64_t>(lim, std::max<int64_t>(1, n_wall - (c.step - rbs)));
        }
        const int chunk = (int)lim;
        int reps = 1;
        if (queued_rebuild) {
            if (c.tune.use_graph) {
                hipGraphExec_t g = nullptr;
                TRY(rebuild_graph_n(c, c.cur, chunk, &g));
                HIPCHK(hipGraphLaunch(g, c.stream));
            } else {
                HIPCHK(enqueue_rebuild(c, nullptr));
                HIPCHK(launch_arm_replay(c.a, c.stream));
                HIPCHK(enqueue_list_steps(c, c.cur, chunk));
            }
        } else if (c.tune.use_graph && chunk == kChunk) {
            TRY(ensure_list_graph(c));
            // plain steps: up to kReplaysPerSync replays per host round trip; a
            // replay queued after one that went stale does nothing (the stale
            // step stays recorded), and kChunk is even, so every replay starts
            // at the same buffer parity
            static_assert(kChunk % 2 == 0, "replays queued back to back share a parity");
            // (as many as the lists are expected to outlast)
            if (!c.cl.mode) {
                const double fit = std::floor(c.rebuild_interval / kChunk);
                reps = (int)std::min<double>({(double)kReplaysPerSync, (double)(left / kChunk),
                                              std::max(1.0, fit)});
            }
            for (int r = 0; r < reps; ++r) {
                if (r > 0)
                    HIPCHK(launch_set_u64((unsigned long long *)c.a.step_base,
                                          (unsigned long long)(c.step + (int64_t)r * kChunk),
                                          c.stream));
                HIPCHK(hipGraphLaunch(c.lgraph[c.cl.plain_launch ? 1 : 0][c.cur], c.stream));
            }
        } else if (c.tune.use_graph) {
            // a shorter replay (a step count below kChunk, the rest of one, or
            // the steps up to a closure check), captured once per length
            hipGraphExec_t g = nullptr;
            TRY(list_graph_n(c, c.cur, chunk, &g));
            HIPCHK(hipGraphLaunch(g, c.stream));
        } else {
            HIPCHK(enqueue_list_steps(c, c.cur, chunk));
        }
        HIPCHK(hipMemcpyAsync(&c.rb->ctl, c.ctl, sizeof(Ctx::Ctl), hipMemcpyDeviceToHost,
                              c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        const unsigned long long inv = c.rb->ctl.inv;
        const int st = c.rb->ctl.st;
        if (queued_rebuild) {
            // lists too short: the replay did nothing; longer lists, rebuilt
            if (c.rb->ctl.over > 0) {
                TRY(grow_lists(c, c.rb->ctl.over));
                continue;
            }
            TRY(rebuild_done(c));
        }
        const int64_t queued = (int64_t)chunk * reps;
        int64_t done = queued;
        if (inv != ~0ull) {
            const int64_t lim = (int64_t)inv - 1 - c.step;  // steps that ran
            done = std::max<int64_t>(0, std::min<int64_t>(queued, lim));
        }
        c.cur = (int)((c.cur + done) & 1);
        c.step += done;
        left -= done;
        if (inv != ~0ull && (int64_t)inv <= c.step + 1) c.list_valid = false;
        if (st) return read_status(c);
    }
    c.cl.plain_launch = true;
    set_state_ptrs(c, c.cur);
    TRY(set_device_step(c));
    return PD_OK;
}

// ---------------------------------------------------------------------------
// modal closure (host side)
// ---------------------------------------------------------------------------
void dfree(Ctx &c, void *p) {
    if (!p) return;
    hipFree(p);
    c.owned.erase(std::remove(c.owned.begin(), c.owned.end(), p), c.owned.end());
}

// Young's modulus behind a micromodulus (Table tab:2d-peri, nu = 1/3)
double young_of(const MatConst &m) {
    const double e3 = m.eps * m.eps * m.eps;
    return m.conic ? m.cw * kPi * e3 * (2.0 / 3.0) / 24.0 : m.cw * kPi * e3 * (2.0 / 3.0) / 6.0;
}

// the reference bonds (both directions) of the particle p, local indices
pd_status particle_bonds(Ctx &c, int p, std::vector<std::pair<int, int>> &out) {
    const int n0 = c.h_poff[p], n1 = c.h_poff[p + 1];
    const int sl0 = n0 / kSlice, sl1 = (n1 - 1) / kSlice + 1;
    const uint32_t w0 = c.h_slice_ptr[sl0], w1 = c.h_slice_ptr[sl1];
    std::vector<uint32_t> col(w1 - w0);
    HIPCHK(hipMemcpyAsync(col.data(), c.a.col + w0, (w1 - w0) * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    out.clear();
    for (int i = n0; i < n1; ++i) {
        const int sl = i / kSlice;
        const uint32_t base = c.h_slice_ptr[sl] - w0 + (uint32_t)(i % kSlice);
        const int W = (int)((c.h_slice_ptr[sl + 1] - c.h_slice_ptr[sl]) / kSlice);
        for (int k = 0; k < W; ++k) {
            const int j = (int)(col[base + (uint32_t)k * kSlice] & kIndexMask);
            if (j == i) continue;  // padding
            if (j < n0 || j >= n1) return fail(c, PD_E_STATE, "bond leaves its particle");
            out.emplace_back(i - n0, j - n0);
        }
    }
    return PD_OK;
}

// largest linear stretch of each mode over the template's bonds
void mode_stretch_bound(const ClState &L, int s, const std::vector<double> &X,
                        const std::vector<double> &Y, double *sig) {
    const std::vector<double> &ph = L.h_phi[s];
    for (int k = 0; k < kClModes; ++k) sig[k] = 0.0;
    for (const auto &b : L.h_tbonds[s]) {
        const int i = b.first, j = b.second;
        const double dx = X[j] - X[i], dy = Y[j] - Y[i];
        const double L2 = dx * dx + dy * dy;
        for (int k = 0; k < kClModes; ++k) {
            const double ex = ph[(j * kClModes + k) * 2] - ph[(i * kClModes + k) * 2];
            const double ey = ph[(j * kClModes + k) * 2 + 1] - ph[(i * kClModes + k) * 2 + 1];
            sig[k] = std::max(sig[k], fabs(ex * dx + ey * dy) / L2);
        }
    }
}

pd_status upload_shape_modes(Ctx &c, int s) {
    ClState &L = c.cl;
    const int n = L.h_shape_n[s];
    std::vector<float> f((size_t)n * 2 * kClModes);
    for (size_t k = 0; k < f.size(); ++k) f[k] = (float)L.h_phi[s][k];
    HIPCHK(hipMemcpyAsync(L.phi + (size_t)L.h_toff[s] * 2 * kClModes, f.data(), f.size() * sizeof(float),
                          hipMemcpyHostToDevice, c.stream));
    // mode-major copy: mode k of template node i at (k * NT + toff + i)
    const size_t NT = (size_t)L.ca.NT;
    for (int k = 0; k < kClModes; ++k) {
        std::vector<float> col((size_t)2 * n);
        for (int i = 0; i < n; ++i) {
            col[2 * i] = f[((size_t)i * kClModes + k) * 2];
            col[2 * i + 1] = f[((size_t)i * kClModes + k) * 2 + 1];
        }
        HIPCHK(hipMemcpyAsync(L.phiT + 2 * ((size_t)k * NT + L.h_toff[s]), col.data(),
                              col.size() * sizeof(float), hipMemcpyHostToDevice, c.stream));
    }
    HIPCHK(hipMemcpyAsync(L.lam + s * kClModes, &L.h_lam[s * kClModes], kClModes * sizeof(double),
                          hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(L.sig + s * kClModes, &L.h_sig[s * kClModes], kClModes * sizeof(double),
                          hipMemcpyHostToDevice, c.stream));
    // reduced mode: b_k = sum m X . phi_k with the modes as the kernels hold
    // them, so that the polar moment is I0 + 2 b.q + q.q
    // and phimax_k = max_i |phi_k(i)|, for the bound on the motion
    if (L.bvec && L.phimax) {
        const int t0 = L.h_toff[s], m0 = c.h_poff[L.h_shape_first[s]];
        std::vector<double> b(kClModes, 0.0), pm(kClModes, 0.0);
        for (int k = 0; k < kClModes; ++k)
            for (int i = 0; i < n; ++i) {
                const double fx = f[((size_t)i * kClModes + k) * 2], fy = f[((size_t)i * kClModes + k) * 2 + 1];
                b[k] += c.h_mass[m0 + i] * (L.h_tX[t0 + i] * fx + L.h_tY[t0 + i] * fy);
                pm[k] = std::max(pm[k], sqrt(fx * fx + fy * fy));
            }
        HIPCHK(hipMemcpyAsync(L.bvec + s * kClModes, b.data(), kClModes * sizeof(double),
                              hipMemcpyHostToDevice, c.stream));
        HIPCHK(hipMemcpyAsync(L.phimax + s * kClModes, pm.data(), kClModes * sizeof(double),
                              hipMemcpyHostToDevice, c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

// stiffness of the linearised bond force of eq. (peri) about the template's
// reference configuration, K = -dF/du; the lowest non-rigid solutions of
// K phi = lambda M phi (M = diag(rho V)), normalised phi^T M phi = 1, each
// signed so that its largest entry is positive
pd_status shape_modes(Ctx &c, int s) {
    ClState &L = c.cl;
    const int pt = L.h_shape_first[s];
    const int n0 = c.h_poff[pt], n = L.h_shape_n[s];
    const MatConst &mc = c.h_mc[c.h_pmat[pt]];
    TRY(particle_bonds(c, pt, L.h_tbonds[s]));
    const int D = 2 * n;
    std::vector<double> K((size_t)D * D, 0.0);
    for (const auto &b : L.h_tbonds[s]) {
        const int i = b.first, j = b.second;
        const double dx = c.h_x[n0 + j] - c.h_x[n0 + i], dy = c.h_y[n0 + j] - c.h_y[n0 + i];
        const double l = sqrt(dx * dx + dy * dy);
        const double ex = dx / l, ey = dy / l;
        const double w = mc.conic ? 1.0 - l / mc.eps : 1.0;
        const double k = mc.cw * w * c.h_vol[n0 + i] * c.h_vol[n0 + j] / l;
        const double e[2] = {ex, ey};
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
                K[(size_t)(2 * i + p) * D + 2 * i + q] += k * e[p] * e[q];
                K[(size_t)(2 * i + p) * D + 2 * j + q] -= k * e[p] * e[q];
            }
    }
    std::vector<double> rs(D);
    for (int i = 0; i < n; ++i) rs[2 * i] = rs[2 * i + 1] = 1.0 / sqrt(c.h_mass[n0 + i]);
    for (int r = 0; r < D; ++r)
        for (int q = 0; q < D; ++q) K[(size_t)r * D + q] *= rs[r] * rs[q];
    std::vector<double> w;
    try {
        sym_eig(K, D, w);
    } catch (const std::exception &ex) {
        return fail(c, PD_E_DEVICE, ex.what());
    }
    const int nm = std::min(kClModes, D - 3);
    if (nm < 1 || !(fabs(w[2]) <= 1e-8 * w[3]))
        return fail(c, PD_E_INVALID, "a closure shape must have exactly three rigid modes");
    L.h_nmodes[s] = nm;
    std::vector<double> &ph = L.h_phi[s];
    ph.assign((size_t)n * 2 * kClModes, 0.0);
    for (int k = 0; k < nm; ++k) {
        const int col = 3 + k;
        double big = 0.0;
        int at = 0;
        for (int r = 0; r < D; ++r) {
            const double v = K[(size_t)r * D + col] * rs[r];
            if (fabs(v) > fabs(big) * (1.0 + 1e-12)) {
                big = v;
                at = r;
            }
        }
        (void)at;
        const double sg = big < 0.0 ? -1.0 : 1.0;
        for (int r = 0; r < D; ++r)
            ph[((size_t)(r / 2) * kClModes + k) * 2 + (r & 1)] = sg * K[(size_t)r * D + col] * rs[r];
        L.h_lam[s * kClModes + k] = w[col];
    }
    for (int k = nm; k < kClModes; ++k) L.h_lam[s * kClModes + k] = 0.0;
    std::vector<double> X(n), Y(n);
    for (int i = 0; i < n; ++i) {
        X[i] = c.h_x[n0 + i];
        Y[i] = c.h_y[n0 + i];
    }
    mode_stretch_bound(L, s, X, Y, &L.h_sig[s * kClModes]);
    return upload_shape_modes(c, s);
}

pd_status closure_setup(Ctx &c, const int32_t *sp, double gate_frac, const double *tau_c,
                        int32_t check_every, double err_tol) {
    ClState &L = c.cl;
    if (L.ready) return fail(c, PD_E_STATE, "the closure is already set up");
    if (!sp) return fail(c, PD_E_INVALID, "missing shape_of_particle");
    if (!(gate_frac > 0.0) || check_every < 0 || !(err_tol > 0.0))
        return fail(c, PD_E_INVALID, "gate_frac and err_tol must be positive, check_every >= 0");
    const int P = c.P;
    int S = 0;
    for (int p = 0; p < P; ++p) {
        if (sp[p] < -1) return fail(c, PD_E_INVALID, "shape ids are -1 (none) or >= 0");
        S = std::max(S, sp[p] + 1);
    }
    if (S == 0) return fail(c, PD_E_INVALID, "no particle has a closure shape");
    L.S = S;
    L.h_shape_first.assign(S, -1);
    L.h_shape_n.assign(S, 0);
    L.h_toff.assign(S, 0);
    L.h_nmodes.assign(S, 0);
    L.h_trained.assign(S, 0);
    L.h_phi.assign(S, {});
    L.h_tbonds.assign(S, {});
    L.h_lam.assign((size_t)S * kClModes, 0.0);
    L.h_sig.assign((size_t)S * kClModes, 0.0);
    L.adam_t.assign(S, 0);
    L.h_cpart.clear();
    L.h_cshape.clear();
    for (int s = 0; s < S; ++s)
        for (int p = 0; p < P; ++p)
            if (sp[p] == s) {
                if (L.h_shape_first[s] < 0) L.h_shape_first[s] = p;
                L.h_cpart.push_back(p);
                L.h_cshape.push_back(s);
            }
    for (int s = 0; s < S; ++s)
        if (L.h_shape_first[s] < 0) return fail(c, PD_E_INVALID, "shape ids must be 0 .. S-1, each used");
    L.Pc = (int)L.h_cpart.size();
    // templates: the first particle of each shape, about its mass centroid
    std::vector<double> tX, tY;
    L.max_n = 0;
    for (int s = 0; s < S; ++s) {
        const int pt = L.h_shape_first[s];
        const int n0 = c.h_poff[pt], n = c.h_poff[pt + 1] - n0;
        if (n > kClMaxNodes || n < 3)
            return fail(c, PD_E_INVALID, "a closure particle has 3 .. 1024 nodes");
        L.h_shape_n[s] = n;
        L.h_toff[s] = (int)tX.size();
        L.max_n = std::max(L.max_n, n);
        double M = 0, sx = 0, sy = 0;
        for (int i = n0; i < n0 + n; ++i) {
            M += c.h_mass[i];
            sx += c.h_mass[i] * c.h_x[i];
            sy += c.h_mass[i] * c.h_y[i];
        }
        for (int i = n0; i < n0 + n; ++i) {
            tX.push_back(c.h_x[i] - sx / M);
            tY.push_back(c.h_y[i] - sy / M);
        }
    }
    // every particle of a shape is its template rotated and translated
    for (int k = 0; k < L.Pc; ++k) {
        const int p = L.h_cpart[k], s = L.h_cshape[k];
        const int n0 = c.h_poff[p], n = c.h_poff[p + 1] - n0;
        const int t0 = L.h_toff[s], q0 = c.h_poff[L.h_shape_first[s]];
        if (n != L.h_shape_n[s]) return fail(c, PD_E_INVALID, "particles of one shape differ in node count");
        double M = 0, sx = 0, sy = 0, rmax = 0;
        for (int i = 0; i < n; ++i) {
            if (fabs(c.h_mass[n0 + i] - c.h_mass[q0 + i]) > 1e-12 * c.h_mass[q0 + i])
                return fail(c, PD_E_INVALID, "particles of one shape differ in nodal mass");
            M += c.h_mass[n0 + i];
            sx += c.h_mass[n0 + i] * c.h_x[n0 + i];
            sy += c.h_mass[n0 + i] * c.h_y[n0 + i];
            rmax = std::max(rmax, hypot(tX[t0 + i], tY[t0 + i]));
        }
        double cr = 0, dt = 0;
        for (int i = 0; i < n; ++i) {
            const double Yx = c.h_x[n0 + i] - sx / M, Yy = c.h_y[n0 + i] - sy / M;
            cr += c.h_mass[n0 + i] * (tX[t0 + i] * Yy - tY[t0 + i] * Yx);
            dt += c.h_mass[n0 + i] * (tX[t0 + i] * Yx + tY[t0 + i] * Yy);
        }
        const double th = atan2(cr, dt), ct = cos(th), st = sin(th);
        for (int i = 0; i < n; ++i) {
            const double Yx = c.h_x[n0 + i] - sx / M, Yy = c.h_y[n0 + i] - sy / M;
            const double rx = ct * tX[t0 + i] - st * tY[t0 + i] - Yx;
            const double ry = st * tX[t0 + i] + ct * tY[t0 + i] - Yy;
            if (hypot(rx, ry) > 1e-9 * rmax)
                return fail(c, PD_E_INVALID, "a particle is not a rigid copy of its shape's first particle");
        }
    }
    // device buffers
    const size_t Pc = L.Pc;
    L.h_tX = tX;
    L.h_tY = tY;
    TRY(upload(c, &L.tX, tX.data(), tX.size()));
    TRY(upload(c, &L.tY, tY.data(), tY.size()));
    // reduced mode: per-shape mass, polar moment and size; buffers of the
    // reduced state and of the active node lists
    {
        std::vector<double> Mt(S), I0(S), rmax(S);
        for (int s = 0; s < S; ++s) {
            const int pt = L.h_shape_first[s];
            const int n0 = c.h_poff[pt], n = L.h_shape_n[s];
            double M = 0.0, I = 0.0, r = 0.0;
            for (int i = 0; i < n; ++i) {
                const double m = c.h_mass[n0 + i];
                const double X = tX[L.h_toff[s] + i], Y = tY[L.h_toff[s] + i];
                M += m;
                I += m * (X * X + Y * Y);
                r = std::max(r, sqrt(X * X + Y * Y));
            }
            Mt[s] = M;
            I0[s] = I;
            rmax[s] = r;
        }
        TRY(upload(c, &L.Mt, Mt.data(), S));
        TRY(upload(c, &L.I0, I0.data(), S));
        TRY(upload(c, &L.rmax, rmax.data(), S));
        TRY(dalloc(c, &L.bvec, (size_t)S * kClModes));
        TRY(dalloc(c, &L.phimax, (size_t)S * kClModes));
        TRY(dalloc(c, &L.rs, Pc * 16));
        TRY(dalloc(c, &L.qr, Pc * kClModes));
        TRY(dalloc(c, &L.qv, Pc * kClModes));
        TRY(dalloc(c, &L.qa, Pc * kClModes));
        TRY(dalloc(c, &L.qrb, Pc * kClModes));
        TRY(dalloc(c, &L.alist, Pc * (size_t)L.max_n));
        TRY(dalloc(c, &L.acnt, Pc));
        TRY(dalloc(c, &L.act, (size_t)c.N));
        HIPCHK(hipMemsetAsync(L.acnt, 0, Pc * sizeof(int), c.stream));
    }
    TRY(dalloc(c, &L.phi, tX.size() * 2 * kClModes));
    TRY(dalloc(c, &L.phiT, tX.size() * 2 * kClModes));
    L.ca.NT = (int)tX.size();
    TRY(dalloc(c, &L.lam, (size_t)S * kClModes));
    TRY(dalloc(c, &L.sig, (size_t)S * kClModes));
    for (int s = 0; s < S; ++s) TRY(shape_modes(c, s));
    std::vector<double> s0(S), tc(S);
    for (int s = 0; s < S; ++s) {
        const int pt = L.h_shape_first[s];
        const MatConst &mc = c.h_mc[c.h_pmat[pt]];
        s0[s] = mc.s0;
        double rmax = 0;
        for (int i = 0; i < L.h_shape_n[s]; ++i)
            rmax = std::max(rmax, hypot(tX[L.h_toff[s] + i], tY[L.h_toff[s] + i]));
        // default contact threshold: the load that strains the particle's
        // diameter by a tenth of the critical stretch
        tc[s] = (tau_c && tau_c[s] > 0.0) ? tau_c[s] : 0.1 * mc.s0 * young_of(mc) * 2.0 * rmax;
    }
    L.h_tau_c = tc;
    TRY(upload(c, &L.s0, s0.data(), S));
    TRY(upload(c, &L.tau_c, tc.data(), S));
    std::vector<int> zeros(c.P, 0);
    TRY(upload(c, &L.on, zeros.data(), c.P));
    int *dcpart, *dcshape;
    TRY(upload(c, &dcpart, L.h_cpart.data(), Pc));
    TRY(upload(c, &dcshape, L.h_cshape.data(), Pc));
    double *red, *q, *gext, *ghat;
    TRY(dalloc(c, &red, Pc * 16));
    TRY(dalloc(c, &q, Pc * kClModes));
    TRY(dalloc(c, &gext, Pc * kClModes));
    TRY(dalloc(c, &ghat, Pc * kClModes));
    TRY(dalloc(c, &L.fx, (size_t)c.N));
    TRY(dalloc(c, &L.fy, (size_t)c.N));
    TRY(dalloc(c, &L.smax, (size_t)c.N));
    TRY(dalloc(c, &L.stats, 4));
    TRY(dalloc(c, &L.per, Pc * 4));
    TRY(dalloc(c, &L.fallbacks, 1));
    HIPCHK(hipMemsetAsync(L.fallbacks, 0, sizeof(unsigned long long), c.stream));
    HIPCHK(hipMemsetAsync(q, 0, Pc * kClModes * sizeof(double), c.stream));
    // MLP parameters: zero (the linear closure) until loaded or trained
    TRY(dalloc(c, &L.wf, (size_t)S * kClParams));
    TRY(dalloc(c, &L.wb, (size_t)S * kClParams));
    HIPCHK(hipMemsetAsync(L.wf, 0, (size_t)S * kClParams * sizeof(float), c.stream));
    HIPCHK(hipMemsetAsync(L.wb, 0, (size_t)S * kClParams * sizeof(uint16_t), c.stream));
    TRY(dalloc(c, &L.wfr, (size_t)S * kClFrag));
    HIPCHK(hipMemsetAsync(L.wfr, 0, (size_t)S * kClFrag * sizeof(uint16_t), c.stream));
    std::vector<float> ones((size_t)S * kClModes, 1.0f);
    TRY(upload(c, &L.sig_q, ones.data(), ones.size()));
    TRY(upload(c, &L.sig_r, ones.data(), ones.size()));
    // 16-row blocks of the MLP, each within one shape
    L.h_rb_shape.clear();
    L.h_rb_first.clear();
    L.h_rb_count.clear();
    for (int k = 0; k < L.Pc;) {
        const int s = L.h_cshape[k];
        int e = k;
        while (e < L.Pc && L.h_cshape[e] == s && e - k < 16) ++e;
        L.h_rb_shape.push_back(s);
        L.h_rb_first.push_back(k);
        L.h_rb_count.push_back(e - k);
        k = e;
    }
    int *rbs, *rbf, *rbc;
    TRY(upload(c, &rbs, L.h_rb_shape.data(), L.h_rb_shape.size()));
    TRY(upload(c, &rbf, L.h_rb_first.data(), L.h_rb_first.size()));
    TRY(upload(c, &rbc, L.h_rb_count.data(), L.h_rb_count.size()));
    int *dtoff;
    TRY(upload(c, &dtoff, L.h_toff.data(), S));
    HIPCHK(hipStreamSynchronize(c.stream));

    ClArgs &ca = L.ca;
    const int NT = ca.NT;
    ca = ClArgs{};
    ca.NT = NT;
    ca.phiT = reinterpret_cast<const float2 *>(L.phiT);
    ca.Pc = L.Pc;
    ca.cpart = dcpart;
    ca.cshape = dcshape;
    ca.poff = c.d_poff;
    ca.toff = dtoff;
    ca.tX = L.tX;
    ca.tY = L.tY;
    ca.phi = L.phi;
    ca.lam = L.lam;
    ca.sig = L.sig;
    ca.s0 = L.s0;
    ca.tau_c = L.tau_c;
    ca.gate_frac = gate_frac;
    ca.learned = 0;
    ca.red = red;
    ca.q = q;
    ca.gext = gext;
    ca.ghat = ghat;
    ca.fallbacks = L.fallbacks;
    ca.rb_shape = rbs;
    ca.rb_first = rbf;
    ca.rb_count = rbc;
    ca.n_rb = (int)L.h_rb_shape.size();
    ca.n_slices = (L.max_n + 31) / 32;
    TRY(dalloc(c, &ca.part, Pc * ca.n_slices * kClModes * 2));
    ca.rs = L.rs;
    ca.qr = L.qr;
    ca.qv = L.qv;
    ca.qa = L.qa;
    ca.qrb = L.qrb;
    ca.alist = L.alist;
    ca.acnt = L.acnt;
    ca.max_n = L.max_n;
    ca.Mt = L.Mt;
    ca.I0 = L.I0;
    ca.bvec = L.bvec;
    ca.phimax = L.phimax;
    ca.rmax = L.rmax;
    MlpArgs &m = L.ma;
    m = MlpArgs{};
    m.rows = L.Pc;
    m.row_blocks = (int)L.h_rb_shape.size();
    m.rb_shape = rbs;
    m.rb_first = rbf;
    m.rb_count = rbc;
    m.q = q;
    m.lam = L.lam;
    m.wb = L.wb;
    m.wfr = L.wfr;
    m.wf = L.wf;
    m.sig_q = L.sig_q;
    m.sig_r = L.sig_r;
    m.g = ghat;
    L.check_every = check_every;
    L.err_tol = err_tol;
    L.ready = true;
    return PD_OK;
}

// the periodic check: plain bond forces (and the largest stretch per node)
// at the current state, the closure's modal force at the same state, and
// the per-particle fallback
pd_status closure_check(Ctx &c) {
    ClState &L = c.cl;
    // smax stays set for the check kernel, which reads it; the force
    // kernels of later steps get it cleared
    c.a.smax = L.smax;
    pd_status st = eval_terms(c);
    if (st == PD_OK) {
        set_state_ptrs(c, c.cur);
        hipError_t e = launch_cl_project(c.a, L.ca, false, 1, L.max_n, c.stream);
        if (e == hipSuccess && L.mode == 2) e = launch_mlp_forward(L.ma, c.a, false, c.stream);
        if (e == hipSuccess) e = launch_cl_check(c.a, L.ca, L.err_tol, L.per, L.stats, c.stream);
        if (e != hipSuccess) st = fail(c, PD_E_DEVICE, hipGetErrorString(e));
    }
    c.a.smax = nullptr;
    TRY(st);
    double r[4];
    HIPCHK(hipMemcpyAsync(r, L.stats, sizeof r, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    ++L.checks;
    L.last_checked = (int64_t)r[3];
    L.last_err = r[1] > 0.0 ? sqrt(r[0] / r[1]) : 0.0;
    L.last_err_linear = r[1] > 0.0 ? sqrt(r[2] / r[1]) : 0.0;
    return PD_OK;
}

pd_status cl_training_buffers(Ctx &c, int rows) {
    ClState &L = c.cl;
    if (!L.t_m) {
        TRY(dalloc(c, &L.t_m, (size_t)L.S * kClParams));
        TRY(dalloc(c, &L.t_v, (size_t)L.S * kClParams));
        TRY(dalloc(c, &L.t_grad, (size_t)kClParams));
    }
    if (L.tcap >= rows) return PD_OK;
    void *bufs[] = {L.t_y, L.t_z1, L.t_z2, L.t_dy, L.t_dz2, L.t_dz1, L.t_xb, L.t_h1, L.t_h2,
                    L.t_dyb, L.t_dz2b, L.t_dz1b, L.t_idx, L.t_part};
    for (void *b : bufs) dfree(c, b);
    const size_t R = rows;
    TRY(dalloc(c, &L.t_y, R * kClModes));
    TRY(dalloc(c, &L.t_z1, R * kClHidden));
    TRY(dalloc(c, &L.t_z2, R * kClHidden));
    TRY(dalloc(c, &L.t_dy, R * kClModes));
    TRY(dalloc(c, &L.t_dz2, R * kClHidden));
    TRY(dalloc(c, &L.t_dz1, R * kClHidden));
    TRY(dalloc(c, &L.t_xb, R * kClModes));
    TRY(dalloc(c, &L.t_h1, R * kClHidden));
    TRY(dalloc(c, &L.t_h2, R * kClHidden));
    TRY(dalloc(c, &L.t_dyb, R * kClModes));
    TRY(dalloc(c, &L.t_dz2b, R * kClHidden));
    TRY(dalloc(c, &L.t_dz1b, R * kClHidden));
    TRY(dalloc(c, &L.t_idx, R));
    TRY(dalloc(c, &L.t_part, R * kClModes / 256 + 1));
    L.tcap = rows;
    return PD_OK;
}

// loss and gradients of one batch (rows of q, g; idx selects them or null)
hipError_t cl_grad_batch(Ctx &c, int s, const double *q, const double *g, int rows, const int *idx,
                         float *loss) {
    ClState &L = c.cl;
    MlpArgs m{};
    m.rows = rows;
    m.row_blocks = (rows + 15) / 16;
    m.shape = s;
    m.idx = idx;
    m.q = q;
    m.lam = L.lam;
    m.wb = L.wb;
    m.wfr = L.wfr;
    m.wf = L.wf;
    m.sig_q = L.sig_q;
    m.sig_r = L.sig_r;
    m.y = L.t_y;
    m.xb = L.t_xb;
    m.h1 = L.t_h1;
    m.h2 = L.t_h2;
    m.z1 = L.t_z1;
    m.z2 = L.t_z2;
    hipError_t e = launch_mlp_forward(m, c.a, false, c.stream);
    if (e == hipSuccess) e = launch_mlp_loss(m, g, L.t_dy, L.t_dyb, L.t_part, loss, c.stream);
    const uint16_t *W = L.wb + (size_t)s * kClParams;
    float *G = L.t_grad;
    const hipStream_t st = c.stream;
    if (e == hipSuccess)
        e = launch_gemm_bf16(kClModes, kClHidden, rows, L.t_dyb, 1, kClModes, L.t_h2, kClHidden, 1,
                             G + kOffW3, kClHidden, 0, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_colsum(L.t_dy, rows, kClModes, G + kOffB3, st);
    if (e == hipSuccess)
        e = launch_gemm_bf16(rows, kClHidden, kClModes, L.t_dyb, kClModes, 1, W + kOffW3, kClHidden, 1,
                             L.t_dz2, kClHidden, 1, L.t_z2, L.t_dz2b, st);
    if (e == hipSuccess)
        e = launch_gemm_bf16(kClHidden, kClHidden, rows, L.t_dz2b, 1, kClHidden, L.t_h1, kClHidden, 1,
                             G + kOffW2, kClHidden, 0, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_colsum(L.t_dz2, rows, kClHidden, G + kOffB2, st);
    if (e == hipSuccess)
        e = launch_gemm_bf16(rows, kClHidden, kClHidden, L.t_dz2b, kClHidden, 1, W + kOffW2, kClHidden,
                             1, L.t_dz1, kClHidden, 1, L.t_z1, L.t_dz1b, st);
    if (e == hipSuccess)
        e = launch_gemm_bf16(kClHidden, kClModes, rows, L.t_dz1b, 1, kClHidden, L.t_xb, kClModes, 1,
                             G + kOffW1, kClModes, 0, nullptr, nullptr, st);
    if (e == hipSuccess) e = launch_colsum(L.t_dz1, rows, kClHidden, G + kOffB1, st);
    return e;
}

// the force workgroups holding nodes of particles under the plain force
pd_status cl_block_list(Ctx &c) {
    ClState &L = c.cl;
    const int B = kSelBlockNodes;
    const int nb = (c.N + B - 1) / B;
    if (L.blk_cap < nb) {
        dfree(c, L.pd_blocks);
        dfree(c, L.blk_listed);
        TRY(dalloc(c, &L.pd_blocks, (size_t)nb));
        TRY(dalloc(c, &L.blk_listed, (size_t)nb));
        L.blk_cap = nb;
    }
    if (!L.n_pd_blocks) TRY(dalloc(c, &L.n_pd_blocks, 1));
    std::vector<int> on(c.P);
    HIPCHK(hipMemcpyAsync(on.data(), L.on, c.P * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    std::vector<int> listed(nb, 0), list;
    for (int p = 0; p < c.P; ++p) {
        if (on[p]) continue;
        const int n0 = c.h_poff[p], n1 = c.h_poff[p + 1];
        for (int b = n0 / B; b <= (n1 - 1) / B; ++b) listed[b] = 1;
    }
    for (int b = 0; b < nb; ++b)
        if (listed[b]) list.push_back(b);
    const int n = (int)list.size();
    if (n) HIPCHK(hipMemcpyAsync(L.pd_blocks, list.data(), n * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(L.blk_listed, listed.data(), nb * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(L.n_pd_blocks, &n, sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    c.a.pd_blocks = L.pd_blocks;
    c.a.n_pd_blocks = L.n_pd_blocks;
    L.ca.pd_blocks = L.pd_blocks;
    L.ca.n_pd_blocks = L.n_pd_blocks;
    L.ca.blk_listed = L.blk_listed;
    L.ca.block_nodes = B;
    return PD_OK;
}

pd_status check_shape(Ctx &c, int s) {
    if (!c.cl.ready) return fail(c, PD_E_STATE, "the closure is not set up");
    if (s < 0 || s >= c.cl.S) return fail(c, PD_E_INVALID, "bad shape id");
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
    if (c.caller_ev) hipEventDestroy(c.caller_ev);
    if (c.rb) hipHostFree(c.rb);
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
    // ---- device, its workspace of pd_forces_noalloc, stream ----
    HIPCHK(hipGetDevice(&c.device));
    HIPCHK(scratch_init(c.device));
    if (p->hip_stream) {
        c.stream = (hipStream_t)p->hip_stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        c.own_stream = true;
        HIPCHK(hipEventCreateWithFlags(&c.caller_ev, hipEventDisableTiming));
    }
    HIPCHK(hipHostMalloc((void **)&c.rb, sizeof(Ctx::Readback), hipHostMallocDefault));
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
    // per aggregate: its particles in order, box, top-wall speed, particle area
    {
        std::vector<int> cnt(A + 1, 0), parts(P);
        for (int q = 0; q < P; ++q) ++cnt[pagg[q] + 1];
        for (int a2 = 0; a2 < A; ++a2) cnt[a2 + 1] += cnt[a2];
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int q = 0; q < P; ++q) parts[fill[pagg[q]]++] = q;
        TRY(upload(c, &c.d_agg_pstart, cnt.data(), A + 1));
        TRY(upload(c, &c.d_agg_parts, parts.data(), P));
        c.h_box.assign(p->box, p->box + 4 * (size_t)A);
        c.h_vtop = vtop;
        c.h_agg_vol.assign(A, 0.0);
        for (int i = 0; i < N; ++i) c.h_agg_vol[pagg[part[i]]] += p->vol[i];
    }
    // kept for the modal-closure setup
    c.h_x.assign(p->x, p->x + N);
    c.h_y.assign(p->y, p->y + N);
    c.h_vol.assign(p->vol, p->vol + N);
    c.h_mass = mass;
    c.h_poff.assign(p->particle_offset, p->particle_offset + P + 1);
    c.h_pmat.assign(p->particle_material, p->particle_material + P);
    c.h_mc = mc;
    c.d_poff = dpoff;
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
            TRY(dalloc(c, &c.UN[b][d], N));
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
    uint8_t *drowfull;
    TRY(dalloc(c, &drowfull, N));
    BondArgs ba{dx, dy, dpart, dpmat, dpoff, dseg, dsegoff, dthr2, N};
    HIPCHK(launch_bonds_count(ba, drowlen, drowfull, c.stream));
    a.row_full = drowfull;
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
    TRY(dalloc(c, &c.hist, (size_t)kRadix * sort_tiles_max(N)));
    TRY(dalloc(c, &c.dtotal, kRadix));
    a.skey = c.skey_buf;
    a.perm = c.perm_buf;
    TRY(dalloc(c, &a.spx, N));
    TRY(dalloc(c, &a.spy, N));
    TRY(dalloc(c, &a.spart, N));
    TRY(dalloc(c, &a.step, 1));
    TRY(dalloc(c, &c.ctl, 1));
    a.invalid_step = &c.ctl->inv;
    a.step_base = &c.ctl->base;
    a.status = &c.ctl->st;
    a.overflow = &c.ctl->over;
    HIPCHK(hipMemsetAsync(c.ctl, 0, sizeof(Ctx::Ctl), c.stream));
    TRY(dalloc(c, &a.clist_n, N));
    TRY(dalloc(c, &a.brk_log, (size_t)16 * N));
    TRY(dalloc(c, &a.node_broken, N));
    TRY(dalloc(c, &a.ubx, N));
    TRY(dalloc(c, &a.uby, N));
    TRY(alloc_lists(c, 16));
    HIPCHK(launch_invalidate(a, ~0ull, c.stream));
    TRY(dalloc(c, &a.counters, C_N));
    HIPCHK(hipMemsetAsync(a.status, 0, sizeof(int), c.stream));
    HIPCHK(hipMemsetAsync(a.counters, 0, sizeof(unsigned long long) * C_N, c.stream));
    c.step = 0;
    TRY(set_device_step(c));
    a.use_lds = c.tune.use_lds;
    a.lanes = c.tune.lanes_per_node;
    TRY(build_windows(c));
    // ---- t = 0: forces at u0, v0 with the break rule; a0 = F / (rho V) + g ----
    HIPCHK(enqueue_search(c, 0, 0, 0));
    set_state_ptrs(c, 0);
    a.ax_o = c.Acc[0][0];
    a.ay_o = c.Acc[0][1];
    HIPCHK(launch_force(a, c.precision, M_PROLOGUE, lds_cap(c), c.stream));
    HIPCHK(launch_node_broken(a, c.stream));  // (the break rule may have broken bonds)
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
    if (on_device) TRY(after_caller(c));
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

pd_status pd_forces_noalloc(pd_ctx *ctx, uint32_t mask, double *fx, double *fy) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!fx || !fy) return fail(c, PD_E_INVALID, "pd_forces_noalloc: null output");
    const size_t need = (size_t)10 * (size_t)c.N * sizeof(double);
    if (need > kScratchBytes)
        return fail(c, PD_E_INVALID,
                    "pd_forces_noalloc: " + std::to_string(c.N) + " nodes need " +
                        std::to_string(need) + " bytes of workspace, more than its " +
                        std::to_string(kScratchBytes) + " (at most " +
                        std::to_string(kScratchBytes / (10 * sizeof(double))) + " nodes)");
    double *ws = scratch_of(c.device);
    if (!ws) return fail(c, PD_E_STATE, "pd_forces_noalloc: no workspace on this device");
    TRY(after_caller(c));
    TRY(rc_sync(c));
    HIPCHK(enqueue_search(c, c.cur, 0, 0));
    set_state_ptrs(c, c.cur);
    DevArgs a = c.a;
    a.terms = ws;       // every entry is written by the force kernel
    a.smax = nullptr;
    HIPCHK(launch_force(a, c.precision, M_FORCES, lds_cap(c), c.stream));
    HIPCHK(launch_sum_terms(a, mask, fx, fy, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_damage(pd_ctx *ctx, double *phi, int64_t *nb, int32_t on_device) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (on_device) TRY(after_caller(c));
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

pd_status pd_observables(pd_ctx *ctx, double *out) {
    if (!ctx || !out) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(rc_sync(c));
    const int A = c.A;
    if (!c.d_split) TRY(dalloc(c, &c.d_split, 8 * (size_t)c.N));
    if (!c.d_obs) TRY(dalloc(c, &c.d_obs, 10 * (size_t)A));
    set_state_ptrs(c, c.cur);
    HIPCHK(launch_observables(c.a, c.d_split, c.d_agg_pstart, c.d_agg_parts, c.d_poff, c.d_obs,
                              c.stream));
    std::vector<double> r(10 * (size_t)A);
    HIPCHK(hipMemcpyAsync(r.data(), c.d_obs, r.size() * sizeof(double), hipMemcpyDeviceToHost,
                          c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const double t = (double)c.step * c.a.dt;
    for (int a = 0; a < A; ++a) {
        double *o = out + 12 * (size_t)a;
        for (int k = 0; k < 8; ++k) o[k] = r[10 * a + k];
        const double *b = &c.h_box[4 * (size_t)a];
        const double ytop = b[3] - c.h_vtop[a] * t;
        o[8] = c.h_agg_vol[a] / ((b[1] - b[0]) * (ytop - b[2]));
        o[9] = r[10 * a + 8];
        o[10] = r[10 * a + 9];
        o[11] = ytop;
    }
    return PD_OK;
}

pd_status pd_particle_damage(pd_ctx *ctx, double *out, int32_t on_device) {
    if (!ctx || !out) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (on_device) {
        TRY(after_caller(c));
        HIPCHK(launch_particle_damage(c.a, c.d_poff, out, c.stream));
    } else {
        if (!c.d_pdamage) TRY(dalloc(c, &c.d_pdamage, (size_t)c.P));
        HIPCHK(launch_particle_damage(c.a, c.d_poff, c.d_pdamage, c.stream));
        HIPCHK(hipMemcpyAsync(out, c.d_pdamage, c.P * sizeof(double), hipMemcpyDeviceToHost,
                              c.stream));
    }
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_fragments(pd_ctx *ctx, int32_t min_nodes, int32_t *label, int32_t *count,
                       int64_t *n_components, int32_t on_device) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (min_nodes < 1) return fail(c, PD_E_INVALID, "pd_fragments: min_nodes must be >= 1");
    const size_t N = (size_t)c.N, P = (size_t)c.P;
    if (!c.d_cc) TRY(dalloc(c, &c.d_cc, 2 * N + P + 4));
    int *L = c.d_cc, *size = c.d_cc + N, *cnt = c.d_cc + 2 * N, *flags = c.d_cc + 2 * N + P;
    if (on_device) TRY(after_caller(c));
    HIPCHK(launch_cc_init(L, c.N, c.stream));
    // each round takes every label to the smallest one within one more hop,
    // so at most N + 1 rounds reach the fixed point
    int changed = 1;
    for (int64_t round = 0; changed; ++round) {
        if (round > (int64_t)N + 1) return fail(c, PD_E_DEVICE, "pd_fragments: labels did not settle");
        HIPCHK(hipMemsetAsync(flags, 0, sizeof(int), c.stream));
        HIPCHK(launch_cc_round(c.a, L, flags, c.stream));
        HIPCHK(hipMemcpyAsync(&changed, flags, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
    }
    HIPCHK(hipMemsetAsync(size, 0, (N + P + 4) * sizeof(int), c.stream));
    HIPCHK(launch_cc_count(c.a, L, size, min_nodes, cnt, flags + 1, c.stream));
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (label && N) HIPCHK(hipMemcpyAsync(label, L, N * sizeof(int), k, c.stream));
    if (count && P) HIPCHK(hipMemcpyAsync(count, cnt, P * sizeof(int), k, c.stream));
    int ncomp = 0;
    HIPCHK(hipMemcpyAsync(&ncomp, flags + 1, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (n_components) *n_components = ncomp;
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
    TRY(rc_sync(c));
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
    TRY(rc_sync(c));
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
        HIPCHK(launch_node_broken(c.a, c.stream));
    }
    c.step = step;
    TRY(set_device_step(c));
    HIPCHK(hipMemsetAsync(c.a.status, 0, sizeof(int), c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    c.status = 0;
    c.list_valid = false;
    c.rebuild_interval = 1e9;
    c.last_rebuild_step = step;
    set_state_ptrs(c, 0);
    if (c.cl.ready && c.cl.mode && c.cl.reduced) {
        // the reduced state of the closure particles from the loaded nodes,
        // which are then put on the rigid + modal motion
        HIPCHK(launch_rc_init(c.a, c.cl.ca, c.stream));
        TRY(rc_sync(c));
        HIPCHK(hipStreamSynchronize(c.stream));
    }
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
    if (!(t->lanes_per_node == 1 || t->lanes_per_node == 2 || t->lanes_per_node == 4))
        return fail(c, PD_E_INVALID, "lanes_per_node must be 1, 2 or 4");
    if (!(t->cell_factor >= 1.0) || t->cell_factor > 64.0)
        return fail(c, PD_E_INVALID, "cell_factor must be in [1, 64]");
    if (!(t->skin_factor >= 0.0) || t->skin_factor > 16.0)
        return fail(c, PD_E_INVALID, "skin_factor must be in [0, 16]");
    if (c.cl.mode && !(t->skin_factor > 0.0))
        return fail(c, PD_E_INVALID, "the modal closure runs with candidate lists (skin_factor > 0)");
    if (!(t->wall_pass == 0 || t->wall_pass == 1))
        return fail(c, PD_E_INVALID, "wall_pass must be 0 or 1");
    HIPCHK(hipStreamSynchronize(c.stream));
    if (t->wall_pass && !c.a.wfx) {
        // the pass's node lists, wall forces and contact sums (kept until the
        // context ends)
        int *wl, *cl;
        unsigned long long *wn, *cn;
        double *fx, *fy, *cs;
        TRY(dalloc(c, &wl, (size_t)c.N));
        TRY(dalloc(c, &wn, 1));
        TRY(dalloc(c, &fx, (size_t)c.N));
        TRY(dalloc(c, &fy, (size_t)c.N));
        TRY(dalloc(c, &cl, (size_t)c.N));
        TRY(dalloc(c, &cn, 1));
        TRY(dalloc(c, &cs, (size_t)4 * c.N));
        c.a.wall_list = wl;
        c.a.wall_n = wn;
        c.a.wfx = fx;
        c.a.wfy = fy;
        c.a.cont_list = cl;
        c.a.cont_n = cn;
        c.a.csum = cs;
    }
    const bool regrid = t->cell_factor != c.tune.cell_factor || t->skin_factor != c.tune.skin_factor;
    const bool rewin = t->block_nodes != c.tune.block_nodes;
    c.tune = *t;
    c.tune.use_lds = t->use_lds ? 1 : 0;
    c.tune.use_graph = t->use_graph ? 1 : 0;
    c.a.use_lds = c.tune.use_lds;
    c.a.lanes = c.tune.lanes_per_node;
    c.list_valid = false;
    c.rebuild_interval = 1e9;  // the skin may have changed
    set_list_params(c);
    if (regrid) {
        std::vector<double> box(4 * (size_t)c.A);
        HIPCHK(hipMemcpy(box.data(), c.a.box, box.size() * sizeof(double), hipMemcpyDeviceToHost));
        // release the old grid arrays
        const void *old[] = {c.a.agg_gx0, c.a.agg_gy0, c.a.agg_ncx, c.a.agg_ncy, c.a.agg_cell0,
                             c.a.cell_start, c.a.cell_end};
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
    std::vector<hipEvent_t> ev(nev), fe(2), we(wall_pass_on(c) ? 3 * kChunk : 0);
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    for (auto &e : fe) HIPCHK(hipEventCreate(&e));
    for (auto &e : we) HIPCHK(hipEventCreate(&e));
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool list = c.tune.skin_factor > 0.0;
    auto add_search = [&](bool with_list) -> pd_status {
        float t;
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        acc[0] += t;
        cnt[0] += 1;
        // with one key per thread the keys kernel counts the first pass's
        // digits itself and that pass launches no histogram kernel: its
        // (empty) interval goes to the keys class
        const bool fused = P > 0 && sort_items(c.N) == 1;
        for (int p = 0; p < P; ++p) {
            hipEvent_t *e = ev.data() + 2 + 4 * p;
            HIPCHK(hipEventElapsedTime(&t, e[0], e[1]));
            if (fused && p == 0) {
                acc[0] += t;
            } else {
                acc[1] += t;
                cnt[1] += 1;
            }
            HIPCHK(hipEventElapsedTime(&t, e[1], e[2]));
            acc[2] += t;
            HIPCHK(hipEventElapsedTime(&t, e[2], e[3]));
            acc[3] += t;
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
            hipGraphExec_t g = nullptr;
            const bool wp = wall_pass_on(c);
            if (c.tune.use_graph && !wp) {
                // the launches as pd_step issues them: one graph replay
                if (run == kChunk) {
                    TRY(ensure_list_graph(c));
                    g = c.lgraph[c.cl.plain_launch ? 1 : 0][c.cur];
                } else {
                    TRY(list_graph_n(c, c.cur, run, &g));
                }
            }
            HIPCHK(hipEventRecord(fe[0], c.stream));
            if (wp) {
                // two kernels per step: each launch bracketed by events (the
                // step kernel's duration, not the replay's time per step)
                for (int k = 0; k < run; ++k) {
                    set_state_ptrs(c, (c.cur + k) & 1);
                    c.a.chunk_k = k;
                    HIPCHK(hipEventRecord(we[3 * k], c.stream));
                    HIPCHK(launch_pass(c.a, c.precision, c.stream));
                    HIPCHK(hipEventRecord(we[3 * k + 1], c.stream));
                    HIPCHK(launch_force(c.a, c.precision, M_STEP, lds_cap(c), c.stream, true, 0, true));
                    HIPCHK(hipEventRecord(we[3 * k + 2], c.stream));
                }
                c.a.chunk_k = 0;
            } else if (g) {
                HIPCHK(hipGraphLaunch(g, c.stream));
            } else {
                HIPCHK(enqueue_list_steps(c, c.cur, run));
            }
            HIPCHK(hipEventRecord(fe[1], c.stream));
            unsigned long long inv = 0;
            HIPCHK(hipMemcpyAsync(&inv, c.a.invalid_step, sizeof(inv), hipMemcpyDeviceToHost, c.stream));
            HIPCHK(hipStreamSynchronize(c.stream));
            int64_t done = run;
            if (inv != ~0ull) done = std::max<int64_t>(0, std::min<int64_t>(run, (int64_t)inv - 1 - c.step));
            if (done == run) {  // only complete runs time the kernel
                float t;
                if (wp) {
                    for (int k = 0; k < run; ++k) {
                        HIPCHK(hipEventElapsedTime(&t, we[3 * k], we[3 * k + 1]));
                        acc[7] += t;
                        HIPCHK(hipEventElapsedTime(&t, we[3 * k + 1], we[3 * k + 2]));
                        acc[5] += t;
                    }
                    cnt[7] += run;
                } else {
                    HIPCHK(hipEventElapsedTime(&t, fe[0], fe[1]));
                    acc[5] += t;
                }
                cnt[5] += run;
            }
            c.cur = (int)((c.cur + done) & 1);
            c.step += done;
            s += std::max<int64_t>(done, 1);
            if (inv != ~0ull && (int64_t)inv <= c.step + 1) c.list_valid = false;
        } else {
            set_state_ptrs(c, c.cur);
            HIPCHK(enqueue_keys_sort(c, 1, ev.data()));
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
    for (auto &e : we) hipEventDestroy(e);
    for (int k = 0; k < std::min(n_out, 8); ++k) {
        ms[k] = cnt[k] ? acc[k] / (double)cnt[k] : 0.0;
        if (launches) launches[k] = cnt[k];
    }
    return read_status(c);
}

pd_status pd_autotune(pd_ctx *ctx, int32_t steps, pd_tuning *chosen) {
    if (!ctx || steps < 1) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (c.status) return (pd_status)c.status;
    if (c.cl.mode) return fail(c, PD_E_STATE, "tune before switching the modal closure on");
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
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // One trial: the saved state and bonds back in place, two warm-up steps,
    // then two windows of n steps; the shorter window counts, so that a list
    // rebuild or a graph's first instantiation in one window does not decide.
    auto trial_ms = [&](const pd_tuning &t, int n, float *ms) -> pd_status {
        TRY(pd_set_tuning(ctx, &t));
        for (int k = 0; k < 6; ++k)
            HIPCHK(hipMemcpyAsync(src[k], save + k * c.N, nb, hipMemcpyDeviceToDevice, c.stream));
        HIPCHK(hipMemcpyAsync(c.a.col, save_col, c.nslots * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                              c.stream));
        HIPCHK(launch_node_broken(c.a, c.stream));
        c.cur = cur0;
        c.step = step0;
        c.list_valid = false;
        c.last_rebuild_step = step0;
        TRY(set_device_step(c));
        TRY(pd_step(ctx, 2));
        *ms = 1e30f;
        for (int w = 0; w < 2; ++w) {
            HIPCHK(hipEventRecord(e0, c.stream));
            TRY(pd_step(ctx, n));
            HIPCHK(hipEventRecord(e1, c.stream));
            HIPCHK(hipEventSynchronize(e1));
            float m = 0;
            HIPCHK(hipEventElapsedTime(&m, e0, e1));
            *ms = std::min(*ms, m);
        }
        return PD_OK;
    };
    const int blocks[3] = {256, 128, 64};
    const int lanes[3] = {4, 2, 1};
    // skin 0 (cell search every step) also tries cells of twice the contact
    // radius: four times fewer cells can take a radix pass off the key sort
    const double skins[5] = {0.0, 0.0, 0.5, 1.0, 2.0};
    const double cells[5] = {1.0, 2.0, 1.0, 1.0, 1.0};
    std::vector<std::pair<float, pd_tuning>> tried;
    auto by_time = [](const std::pair<float, pd_tuning> &p, const std::pair<float, pd_tuning> &q) {
        return p.first < q.first;
    };
    pd_status result = PD_OK;
    constexpr int kGrid = 3 * 5 * 2 * 3;
    for (int trial = 0; trial < kGrid && result == PD_OK; ++trial) {
        const int bi = trial / 30, ci = (trial / 6) % 5, li = (trial / 3) % 2, ni = trial % 3;
        // the lane count matters to the list-mode step only
        if (skins[ci] == 0.0 && ni > 0) continue;
        pd_tuning t = base;
        t.block_nodes = blocks[bi];
        t.cell_factor = cells[ci];
        t.skin_factor = skins[ci];
        t.use_lds = 1 - li;
        t.lanes_per_node = skins[ci] > 0.0 ? lanes[ni] : 4;
        t.wall_pass = 0;
        float ms = 0;
        if ((result = trial_ms(t, steps, &ms)) == PD_OK) tried.emplace_back(ms, t);
    }
    // the pass of walls and contact candidates on the three fastest list-mode
    // candidates, then the four fastest of all again over windows three times
    // as long
    if (result == PD_OK) {
        std::stable_sort(tried.begin(), tried.end(), by_time);
        std::vector<std::pair<float, pd_tuning>> with_pass;
        for (size_t k = 0; k < tried.size() && with_pass.size() < 3 && result == PD_OK; ++k) {
            if (!(tried[k].second.skin_factor > 0.0)) continue;
            pd_tuning t = tried[k].second;
            t.wall_pass = 1;
            float ms = 0;
            if ((result = trial_ms(t, steps, &ms)) == PD_OK) with_pass.emplace_back(ms, t);
        }
        tried.insert(tried.end(), with_pass.begin(), with_pass.end());
        std::stable_sort(tried.begin(), tried.end(), by_time);
    }
    float best_ms = 1e30f;
    for (size_t k = 0; k < std::min<size_t>(tried.size(), 4) && result == PD_OK; ++k) {
        float ms = 0;
        if ((result = trial_ms(tried[k].second, 3 * steps, &ms)) != PD_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = tried[k].second;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    pd_status s2 = pd_set_tuning(ctx, &best);
    for (int k = 0; k < 6; ++k)
        HIPCHK(hipMemcpyAsync(src[k], save + k * c.N, nb, hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(c.a.col, save_col, c.nslots * sizeof(uint32_t), hipMemcpyDeviceToDevice, c.stream));
    HIPCHK(launch_node_broken(c.a, c.stream));
    HIPCHK(hipMemcpyAsync(c.a.counters, cnt_save, sizeof cnt_save, hipMemcpyHostToDevice, c.stream));
    c.cur = cur0;
    c.step = step0;
    c.last_rebuild_step = step0;
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

// ---- modal closure ----------------------------------------------------------
pd_status pd_closure_setup(pd_ctx *ctx, const int32_t *shape_of_particle, double gate_frac,
                           const double *tau_c, int32_t check_every, double err_tol) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    HIPCHK(hipStreamSynchronize(c.stream));
    return closure_setup(c, shape_of_particle, gate_frac, tau_c, check_every, err_tol);
}

pd_status pd_closure_modes(pd_ctx *ctx, int32_t shape, int32_t *n_nodes, int32_t *n_modes,
                           double *phi, double *lam, double *sig) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    const ClState &L = c.cl;
    if (n_nodes) *n_nodes = L.h_shape_n[shape];
    if (n_modes) *n_modes = L.h_nmodes[shape];
    if (phi) std::copy(L.h_phi[shape].begin(), L.h_phi[shape].end(), phi);
    if (lam) std::copy(&L.h_lam[shape * kClModes], &L.h_lam[shape * kClModes] + kClModes, lam);
    if (sig) std::copy(&L.h_sig[shape * kClModes], &L.h_sig[shape * kClModes] + kClModes, sig);
    return PD_OK;
}

pd_status pd_closure_set_modes(pd_ctx *ctx, int32_t shape, const double *phi, const double *lam) {
    if (!ctx || !phi || !lam) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    ClState &L = c.cl;
    const int n = L.h_shape_n[shape];
    L.h_phi[shape].assign(phi, phi + (size_t)n * 2 * kClModes);
    for (int k = 0; k < kClModes; ++k) L.h_lam[shape * kClModes + k] = lam[k];
    const int pt = L.h_shape_first[shape], n0 = c.h_poff[pt];
    std::vector<double> X(c.h_x.begin() + n0, c.h_x.begin() + n0 + n);
    std::vector<double> Y(c.h_y.begin() + n0, c.h_y.begin() + n0 + n);
    mode_stretch_bound(L, shape, X, Y, &L.h_sig[shape * kClModes]);
    return upload_shape_modes(c, shape);
}

pd_status pd_closure_load(pd_ctx *ctx, int32_t shape, const float *params, const float *sig_q,
                          const float *sig_r) {
    if (!ctx || !params) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    ClState &L = c.cl;
    float *w = L.wf + (size_t)shape * kClParams;
    HIPCHK(hipMemcpyAsync(w, params, kClParams * sizeof(float), hipMemcpyHostToDevice, c.stream));
    HIPCHK(launch_f32_to_bf16(w, L.wb + (size_t)shape * kClParams, kClParams, c.stream));
    HIPCHK(launch_mlp_pack(L.wb + (size_t)shape * kClParams, L.wfr + (size_t)shape * kClFrag,
                           c.stream));
    if (sig_q)
        HIPCHK(hipMemcpyAsync(L.sig_q + shape * kClModes, sig_q, kClModes * sizeof(float),
                              hipMemcpyHostToDevice, c.stream));
    if (sig_r)
        HIPCHK(hipMemcpyAsync(L.sig_r + shape * kClModes, sig_r, kClModes * sizeof(float),
                              hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    L.h_trained[shape] = 1;
    return PD_OK;
}

pd_status pd_closure_get(pd_ctx *ctx, int32_t shape, float *params, float *sig_q, float *sig_r) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    ClState &L = c.cl;
    if (params)
        HIPCHK(hipMemcpyAsync(params, L.wf + (size_t)shape * kClParams, kClParams * sizeof(float),
                              hipMemcpyDeviceToHost, c.stream));
    if (sig_q)
        HIPCHK(hipMemcpyAsync(sig_q, L.sig_q + shape * kClModes, kClModes * sizeof(float),
                              hipMemcpyDeviceToHost, c.stream));
    if (sig_r)
        HIPCHK(hipMemcpyAsync(sig_r, L.sig_r + shape * kClModes, kClModes * sizeof(float),
                              hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_closure_enable(pd_ctx *ctx, int32_t mode) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!c.cl.ready) return fail(c, PD_E_STATE, "the closure is not set up");
    const bool reduced = (mode & PD_CLOSURE_REDUCED) != 0;
    mode &= ~PD_CLOSURE_REDUCED;
    if (mode < 0 || mode > 2)
        return fail(c, PD_E_INVALID, "mode is 0 (off), 1 (linear) or 2 (learned), optionally | PD_CLOSURE_REDUCED");
    if (mode && !(c.tune.skin_factor > 0.0))
        return fail(c, PD_E_INVALID, "the modal closure runs with candidate lists (skin_factor > 0)");
    ClState &L = c.cl;
    TRY(rc_sync(c));  // leaving a reduced mode: the nodes first
    HIPCHK(hipStreamSynchronize(c.stream));
    std::vector<int> on(c.P, 0);
    if (mode)
        for (int p : L.h_cpart) on[p] = 1;
    HIPCHK(hipMemcpyAsync(L.on, on.data(), c.P * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    L.mode = mode;
    L.reduced = mode && reduced;
    L.ca.learned = mode == 2 ? 1 : 0;
    c.a.cl_on = mode ? L.on : nullptr;
    c.a.cl_fx = L.fx;
    c.a.cl_fy = L.fy;
    if (mode) TRY(cl_block_list(c));
    if (L.reduced) {
        // the reduced state from the current nodes, which are then put on the
        // rigid + modal motion; lists are rebuilt (the guard needs them)
        set_state_ptrs(c, c.cur);
        HIPCHK(launch_rc_init(c.a, L.ca, c.stream));
        TRY(rc_sync(c));
        c.list_valid = false;
    }
    L.last_check_step = c.step;
    invalidate_graph(c);
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_closure_snapshot(pd_ctx *ctx, double *q, double *g, int32_t on_device) {
    if (!ctx || !q || !g) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!c.cl.ready) return fail(c, PD_E_STATE, "the closure is not set up");
    ClState &L = c.cl;
    if (on_device) TRY(after_caller(c));
    TRY(eval_terms(c));
    set_state_ptrs(c, c.cur);
    HIPCHK(launch_cl_project(c.a, L.ca, false, 2, L.max_n, c.stream));
    const size_t nb = (size_t)L.Pc * kClModes * sizeof(double);
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(q, L.ca.q, nb, k, c.stream));
    HIPCHK(hipMemcpyAsync(g, L.ca.gext, nb, k, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return PD_OK;
}

pd_status pd_closure_forward(pd_ctx *ctx, int32_t shape, const double *q, double *g, int64_t n,
                             int32_t on_device) {
    if (!ctx || !q || !g || n < 0 || n > (1 << 24)) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    if (n == 0) return PD_OK;
    ClState &L = c.cl;
    if (on_device) TRY(after_caller(c));
    const double *dq = q;
    double *dg = g, *tq = nullptr, *tg = nullptr;
    const size_t nb = (size_t)n * kClModes * sizeof(double);
    if (!on_device) {
        TRY(dalloc(c, &tq, (size_t)n * kClModes));
        TRY(dalloc(c, &tg, (size_t)n * kClModes));
        HIPCHK(hipMemcpyAsync(tq, q, nb, hipMemcpyHostToDevice, c.stream));
        dq = tq;
        dg = tg;
    }
    MlpArgs m{};
    m.rows = (int)n;
    m.row_blocks = (int)((n + 15) / 16);
    m.shape = shape;
    m.q = dq;
    m.lam = L.lam;
    m.wb = L.wb;
    m.wfr = L.wfr;
    m.wf = L.wf;
    m.sig_q = L.sig_q;
    m.sig_r = L.sig_r;
    m.g = dg;
    HIPCHK(launch_mlp_forward(m, c.a, false, c.stream));
    if (!on_device) HIPCHK(hipMemcpyAsync(g, tg, nb, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    dfree(c, tq);
    dfree(c, tg);
    return PD_OK;
}

pd_status pd_closure_grads(pd_ctx *ctx, int32_t shape, const double *q, const double *g, int64_t n,
                           float *grads, double *loss) {
    if (!ctx || !q || !g || !grads || n < 1 || n > (1 << 20)) return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    ClState &L = c.cl;
    TRY(cl_training_buffers(c, (int)n));
    double *dq, *dg;
    float *dl;
    TRY(dalloc(c, &dq, (size_t)n * kClModes));
    TRY(dalloc(c, &dg, (size_t)n * kClModes));
    TRY(dalloc(c, &dl, 1));
    const size_t nb = (size_t)n * kClModes * sizeof(double);
    HIPCHK(hipMemcpyAsync(dq, q, nb, hipMemcpyHostToDevice, c.stream));
    HIPCHK(hipMemcpyAsync(dg, g, nb, hipMemcpyHostToDevice, c.stream));
    HIPCHK(cl_grad_batch(c, shape, dq, dg, (int)n, nullptr, dl));
    float lf = 0.0f;
    HIPCHK(hipMemcpyAsync(grads, L.t_grad, kClParams * sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&lf, dl, sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (loss) *loss = lf;
    dfree(c, dq);
    dfree(c, dg);
    dfree(c, dl);
    return PD_OK;
}

pd_status pd_closure_train(pd_ctx *ctx, int32_t shape, const double *q, const double *g, int64_t n,
                           int32_t iters, int32_t batch, double lr, uint64_t seed, float *loss_out) {
    if (!ctx || !q || !g || n < 1 || iters < 1 || batch < 16 || batch > (1 << 16) || !(lr > 0.0))
        return PD_E_INVALID;
    Ctx &c = ctx->c;
    TRY(check_shape(c, shape));
    ClState &L = c.cl;
    TRY(after_caller(c));
    TRY(cl_training_buffers(c, batch));
    float *dl;
    TRY(dalloc(c, &dl, (size_t)iters));
    const size_t P = kClParams;
    float *w = L.wf + shape * P;
    uint16_t *wb = L.wb + shape * P;
    float *mo = L.t_m + shape * P, *ve = L.t_v + shape * P;
    // normalisation from the data: rms of the inputs and of the targets
    HIPCHK(launch_norm_stats(q, g, L.lam + shape * kClModes, n, L.sig_q + shape * kClModes,
                             L.sig_r + shape * kClModes, c.stream));
    uint16_t *wfr = L.wfr + shape * (size_t)kClFrag;
    if (!L.h_trained[shape]) {
        HIPCHK(launch_mlp_init(w, wb, seed, c.stream));
        HIPCHK(launch_mlp_pack(wb, wfr, c.stream));
    }
    if (L.adam_t[shape] == 0) {
        HIPCHK(hipMemsetAsync(mo, 0, P * sizeof(float), c.stream));
        HIPCHK(hipMemsetAsync(ve, 0, P * sizeof(float), c.stream));
    }
    const float b1 = 0.9f, b2 = 0.999f;
    for (int it = 0; it < iters; ++it) {
        HIPCHK(launch_batch_idx(L.t_idx, batch, n, seed, it + L.adam_t[shape], c.stream));
        HIPCHK(cl_grad_batch(c, shape, q, g, batch, L.t_idx, dl + it));
        const int64_t t = ++L.adam_t[shape];
        // cosine decay of the step size over this call
        const double lrt = 0.5 * lr * (1.0 + cos(kPi * (double)it / (double)iters));
        const float c1 = (float)(1.0 - pow((double)b1, (double)t));
        const float c2 = (float)(1.0 - pow((double)b2, (double)t));
        HIPCHK(launch_adam(w, wb, L.t_grad, mo, ve, kClParams, (float)lrt, b1, b2, 1e-8f, c1, c2,
                           c.stream));
        HIPCHK(launch_mlp_pack(wb, wfr, c.stream));
    }
    if (loss_out)
        HIPCHK(hipMemcpyAsync(loss_out, dl, iters * sizeof(float), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    dfree(c, dl);
    L.h_trained[shape] = 1;
    return PD_OK;
}

pd_status pd_closure_check(pd_ctx *ctx) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!c.cl.ready || !c.cl.mode) return fail(c, PD_E_STATE, "the closure is not on");
    TRY(closure_check(c));
    c.cl.last_check_step = c.step;
    return PD_OK;
}

pd_status pd_closure_stats(pd_ctx *ctx, double out[8]) {
    if (!ctx || !out) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!c.cl.ready) return fail(c, PD_E_STATE, "the closure is not set up");
    ClState &L = c.cl;
    std::vector<int> on(c.P);
    unsigned long long fb = 0;
    HIPCHK(hipMemcpyAsync(on.data(), L.on, c.P * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(&fb, L.fallbacks, sizeof fb, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    int act = 0;
    for (int p : L.h_cpart) act += on[p] ? 1 : 0;
    out[0] = L.Pc;
    out[1] = act;
    out[2] = (double)fb;
    out[3] = (double)L.checks;
    out[4] = L.last_err;
    out[5] = L.last_err_linear;
    out[6] = (double)L.last_checked;
    out[7] = L.S;
    return PD_OK;
}

pd_status pd_closure_particles(pd_ctx *ctx, int32_t *particle, int32_t *shape, int32_t *active) {
    if (!ctx) return PD_E_INVALID;
    Ctx &c = ctx->c;
    if (!c.cl.ready) return fail(c, PD_E_STATE, "the closure is not set up");
    ClState &L = c.cl;
    std::vector<int> on(c.P);
    HIPCHK(hipMemcpyAsync(on.data(), L.on, c.P * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    for (int k = 0; k < L.Pc; ++k) {
        if (particle) particle[k] = L.h_cpart[k];
        if (shape) shape[k] = L.h_cshape[k];
        if (active) active[k] = on[L.h_cpart[k]];
    }
    return PD_OK;
}

}  // extern "C"
