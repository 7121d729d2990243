// pd_kernels.hip -- gfx950 kernels of libpd.
//
// One pass of the step (Algorithm alg:buildtree of the paper) is:
//   k_keys     cell key of every node at its advanced position
//              u + dt v + dt^2/2 a (velocity-Verlet position update);
//   k_hist / k_digit_scan / k_scatter (x radix passes)
//              stable LSD radix sort of (cell key, node) with 8-bit digits;
//              within a wavefront equal digits are ranked with eight ballots;
//   k_cells    first sorted position of every occupied cell, positions and
//              particle ids in sorted order, step counter;
//   k_force    per node, in a fixed order: contact with the nodes of the 3x3
//              neighbouring cells (repulsion, damping, friction, self-contact),
//              the four walls and their corners, the peridynamic bonds of its
//              SELL-64 row (partners staged in LDS), then the velocity-Verlet
//              velocity update and the advanced displacement.
// Every sum is a gather in a fixed order: no floating-point atomics, so runs
// are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "pd_internal.h"
#include "pd_closure_dev.h"
#include "pd_mlp_dev.h"

namespace pd {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void advanced_pos(const DevArgs &a, int j, bool adv, double &px,
                                             double &py, double &ux, double &uy) {
    ux = a.ux[j];
    uy = a.uy[j];
    if (adv) {  // u + dt v + dt^2/2 a, evaluated left to right without contraction
        ux = (ux + a.dt * a.vx[j]) + a.hdt2 * a.ax[j];
        uy = (uy + a.dt * a.vy[j]) + a.hdt2 * a.ay[j];
    }
    px = a.x[j] + ux;
    py = a.y[j] + uy;
}

// the same advanced displacement and position, read from the previous launch
// of the replay (un) or evaluated (bitwise the same value either way)
__device__ __forceinline__ void advanced_pos_un(const DevArgs &a, int j, bool un, double &px,
                                                double &py, double &ux, double &uy) {
    if (un) {
        ux = a.unx[j];
        uy = a.uny[j];
        px = a.x[j] + ux;
        py = a.y[j] + uy;
    } else {
        advanced_pos(a, j, true, px, py, ux, uy);
    }
}

__device__ __forceinline__ void cell_of(const DevArgs &a, int ag, double px, double py, int &cx,
                                        int &cy) {
    const int ncx = a.agg_ncx[ag], ncy = a.agg_ncy[ag];
    double fx = floor((px - a.agg_gx0[ag]) * a.inv_cell);
    double fy = floor((py - a.agg_gy0[ag]) * a.inv_cell);
    fx = fmin(fmax(fx, 0.0), (double)(ncx - 1));  // fmax drops NaN
    fy = fmin(fmax(fy, 0.0), (double)(ncy - 1));
    cx = (int)fx;
    cy = (int)fy;
}

__device__ __forceinline__ void count(const DevArgs &a, int k, unsigned long long v = 1) {
    if (a.counting && v) atomicAdd(&a.counters[k], v);
}

// 1/x and 1/sqrt(x) in FP64 from the hardware estimates and one Newton step.
// Measured on gfx950 over x in [e^-30, e^-10] (10^6 seeded values): the
// estimates are within 5.2e-8 (rsq) and 4.6e-8 (rcp) relative, one step
// takes them to 4.1e-15 and 2.1e-15 (the quadratic convergence of Newton's
// method from ~2^-24).  The bond force then carries ~1e-14 relative error,
// two orders below the 1e-12 force bar; break decisions do not depend on it
// (a stretch within 1e-10 of s0 is re-decided exactly).
__device__ __forceinline__ double rcp_nr(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsq_nr(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    return fma(r, fma(-0.5 * x * r, r, 0.5), r);
}

// sqrt(x) from the 1/sqrt estimate r: h = x r, refined by one Newton step
// for the square root, h + (h / 2)(1 - h r) (same accuracy as above)
__device__ __forceinline__ double sqrt_nr(double x) {
    const double r = __builtin_amdgcn_rsq(x);
    const double h = x * r;
    return fma(0.5 * h, fma(-h, r, 1.0), h);
}

// inclusive scan across a 64-lane wavefront
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over a 256-thread block; returns the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *total,
                                                       uint32_t *sh /*[4]*/) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t s = sh[q];
        if (q < w) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---------------------------------------------------------------------------
// setup: reference bonds (Algorithm alg:buildtree, reference neighbours) minus
// the non-bonds of Sec. 5.  A candidate bond is dropped when it properly
// crosses a barrier segment of its particle: an edge of the boundary pushed
// outward by delta along the exterior-angle bisectors, or the bisector ray
// of a non-convex vertex up to its first hit with the boundary.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx,
                                         double cy) {
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// A barrier segment that lies along the bond's line (both of its ends within
// rounding of that line, e.g. a bond along the bisector ray of a cusp whose
// vertex is the bond's end node) does not cross it properly; the signs of
// such orientations are rounding noise and would differ between the two
// directions of one bond.
__device__ bool crosses_barrier(double ax, double ay, double bx, double by, const double *seg,
                                int s0, int s1) {
    const double lab = fabs(bx - ax) + fabs(by - ay);
    for (int s = s0; s < s1; ++s) {
        const double cx = seg[4 * s], cy = seg[4 * s + 1], dx = seg[4 * s + 2], dy = seg[4 * s + 3];
        const double o1 = orient(ax, ay, bx, by, cx, cy), o2 = orient(ax, ay, bx, by, dx, dy);
        if (!((o1 > 0.0 && o2 < 0.0) || (o1 < 0.0 && o2 > 0.0))) continue;
        const double tol = 1e-10 * lab * (fabs(dx - cx) + fabs(dy - cy));
        if (fabs(o1) <= tol && fabs(o2) <= tol) continue;  // collinear
        const double o3 = orient(cx, cy, dx, dy, ax, ay), o4 = orient(cx, cy, dx, dy, bx, by);
        if ((o3 > 0.0 && o4 < 0.0) || (o3 < 0.0 && o4 > 0.0)) return true;
    }
    return false;
}

// row lengths; row_full[i]: the line-of-sight filter left out none of the
// node's same-particle neighbours within eps
__global__ void k_bonds_count_w(BondArgs b, int *rowlen, uint8_t *row_full) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.N) return;
    const int p = b.part[i];
    const double thr2 = b.thr2[b.pmat[p]];
    const double xi = b.x[i], yi = b.y[i];
    const double rx = b.x[b.poff[p]], ry = b.y[b.poff[p]];  // particle frame origin
    const int s0 = b.seg_off[p], s1 = b.seg_off[p + 1];
    int n = 0, nall = 0;
    for (int j = b.poff[p]; j < b.poff[p + 1]; ++j) {
        if (j == i) continue;
        const double dx = b.x[j] - xi, dy = b.y[j] - yi;
        const double d2 = dx * dx + dy * dy;
        if (!(d2 < thr2)) continue;
        ++nall;
        if (s1 > s0 && crosses_barrier(xi - rx, yi - ry, b.x[j] - rx, b.y[j] - ry, b.seg, s0, s1))
            continue;
        ++n;
    }
    rowlen[i] = n;
    row_full[i] = n == nall ? 1 : 0;
}

// node_broken[i]: one of the node's bonds is broken (after the bond states
// were set wholesale: at t = 0, a restored state)
__global__ void k_node_broken(DevArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const uint32_t base = a.slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
    const int n = a.rowlen[i];
    uint8_t any = 0;
    for (int k = 0; k < n; ++k) any |= (a.col[base + (uint32_t)k * kSlice] & kBroken) ? 1 : 0;
    a.node_broken[i] = any;
}

__global__ void k_bonds_fill_w(BondArgs b, uint32_t *col, const uint32_t *slice_ptr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= b.N) return;
    const int p = b.part[i];
    const double thr2 = b.thr2[b.pmat[p]];
    const double xi = b.x[i], yi = b.y[i];
    const double rx = b.x[b.poff[p]], ry = b.y[b.poff[p]];  // particle frame origin
    const int s0 = b.seg_off[p], s1 = b.seg_off[p + 1];
    const uint32_t base = slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
    const int W = (int)((slice_ptr[i / kSlice + 1] - slice_ptr[i / kSlice]) / kSlice);
    int n = 0;
    for (int j = b.poff[p]; j < b.poff[p + 1] && n < W; ++j) {
        if (j == i) continue;
        const double dx = b.x[j] - xi, dy = b.y[j] - yi;
        const double d2 = dx * dx + dy * dy;
        if (!(d2 < thr2)) continue;
        if (s1 > s0 && crosses_barrier(xi - rx, yi - ry, b.x[j] - rx, b.y[j] - ry, b.seg, s0, s1))
            continue;
        col[base + (uint32_t)n * kSlice] = (uint32_t)j;
        ++n;
    }
    for (int k = n; k < W; ++k) col[base + (uint32_t)k * kSlice] = (uint32_t)i | kBroken;
}

// staging window of each force block: [min, max] of its nodes and partners
__global__ void k_windows(const uint32_t *col, const uint32_t *slice_ptr, const int *rowlen, int N,
                          int block_nodes, int *win_lo, int *win_hi) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint32_t base = slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
    int lo = i, hi = i;
    for (int k = 0; k < rowlen[i]; ++k) {
        const int j = (int)(col[base + (uint32_t)k * kSlice] & kIndexMask);
        lo = min(lo, j);
        hi = max(hi, j);
    }
    atomicMin(&win_lo[i / block_nodes], lo);
    atomicMax(&win_hi[i / block_nodes], hi);
}

// ---------------------------------------------------------------------------
// cell keys
// ---------------------------------------------------------------------------
// With `hist` set, the workgroup also counts the low digit of its 256 keys:
// when the radix sort takes one key per thread, these workgroups are exactly
// the first pass's tiles, and that pass needs no histogram launch of its own.
static_assert(kRadix == 256, "k_keys counts one digit per thread of a 256-thread workgroup");
__global__ __launch_bounds__(256) void k_keys(DevArgs a, int adv, uint32_t *hist, int G) {
    __shared__ uint32_t cnt[kRadix];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (hist) cnt[threadIdx.x] = 0;
    uint32_t key = 0;
    if (i < a.N) {
        double px, py, ux, uy;
        advanced_pos(a, i, adv != 0, px, py, ux, uy);
        const int ag = a.pagg[a.part[i]];
        int cx, cy;
        cell_of(a, ag, px, py, cx, cy);
        key = a.agg_cell0[ag] + (uint32_t)cy * (uint32_t)a.agg_ncx[ag] + (uint32_t)cx;
        a.keys[i] = key;
    }
    if (hist) {  // uniform: a kernel argument
        __syncthreads();
        if (i < a.N) atomicAdd(&cnt[key & (kRadix - 1)], 1u);
        __syncthreads();
        hist[threadIdx.x * G + blockIdx.x] = cnt[threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// radix sort: histogram, per-digit scan over tiles, stable scatter
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSortBlock) void k_hist(const uint32_t *keys, int N, int shift,
                                                     uint32_t *hist, int G, int items) {
    __shared__ uint32_t cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kSortBlock * items;
    // the tile's keys, all loaded before the first count (one memory round trip)
    uint32_t kr[kSortItemsMax];
#pragma unroll
    for (int r = 0; r < kSortItemsMax; ++r) {
        const int idx = base + r * kSortBlock + threadIdx.x;
        kr[r] = (r < items && idx < N) ? keys[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortItemsMax; ++r) {
        const int idx = base + r * kSortBlock + threadIdx.x;
        if (r < items && idx < N) atomicAdd(&cnt[(kr[r] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * G + blockIdx.x] = cnt[threadIdx.x];
}

// one block per digit: exclusive scan of the digit's tile counts, digit total
__global__ __launch_bounds__(kSortBlock) void k_digit_scan(uint32_t *hist, int G,
                                                           uint32_t *dtotal) {
    __shared__ uint32_t sh[4];
    const int d = blockIdx.x;
    uint32_t carry = 0;
    for (int s = 0; s < G; s += kSortBlock) {
        const int k = s + threadIdx.x;
        const uint32_t v = k < G ? hist[d * G + k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan256(v, &tot, sh);
        if (k < G) hist[d * G + k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) dtotal[d] = carry;
}

__global__ __launch_bounds__(kSortBlock) void k_scatter(const uint32_t *kin, const int *vin,
                                                        uint32_t *kout, int *vout, int N,
                                                        int shift, const uint32_t *hist, int G,
                                                        const uint32_t *dtotal, int items) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wc[4][kRadix];
    __shared__ uint32_t sh[4];
    const int t = threadIdx.x, w = t >> 6;
    const int base = blockIdx.x * kSortBlock * items;
    // the tile's keys and payloads, loaded up front: the rounds below are
    // serialised by barriers, so loads issued inside them would cost one
    // memory round trip each
    uint32_t kr[kSortItemsMax];
    int vr[kSortItemsMax];
#pragma unroll
    for (int r = 0; r < kSortItemsMax; ++r) {
        const int idx = base + r * kSortBlock + t;
        const bool valid = r < items && idx < N;
        kr[r] = valid ? kin[idx] : 0u;
        vr[r] = valid ? (vin ? vin[idx] : idx) : 0;
    }
    uint32_t tot;
    const uint32_t dbase = block_excl_scan256(dtotal[t], &tot, sh);
    run[t] = dbase + hist[t * G + blockIdx.x];
    wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
    __syncthreads();
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int r = 0; r < kSortItemsMax; ++r) {
        if (r >= items) break;  // uniform: a kernel argument
        const int idx = base + r * kSortBlock + t;
        const bool valid = idx < N;
        const uint32_t key = kr[r];
        const int val = vr[r];
        const uint32_t d = (key >> shift) & (kRadix - 1);
        // lanes of this wavefront holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wc[q][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        wc[0][t] = wc[1][t] = wc[2][t] = wc[3][t] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// cell starts and sorted payload
// ---------------------------------------------------------------------------
__global__ void k_cells(DevArgs a, int adv, int advance_step) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (advance_step && k == 0) *a.step += 1;
    if (k >= a.N) return;
    const uint32_t key = a.skey[k];
    if (k == 0 || a.skey[k - 1] != key) a.cell_start[key] = (uint32_t)k;
    if (k == a.N - 1 || a.skey[k + 1] != key) a.cell_end[key] = (uint32_t)k + 1u;
    const int j = a.perm[k];
    double px, py, ux, uy;
    advanced_pos(a, j, adv != 0, px, py, ux, uy);
    a.spx[k] = px;
    a.spy[k] = py;
    a.spart[k] = a.part[j];
}

// ---------------------------------------------------------------------------
// contact laws (Sec. 4.1-4.4) and walls (Sec. 4.5), FP64
// ---------------------------------------------------------------------------
// damping (Sec. 4.3) and friction (Sec. 4.2) on node i; e from i toward the
// partner, vr = v_i - v_partner, Fr = |F_r|, mi = rho_i V_i, Vp = partner
// volume or wall-region area, Kd = stiffness in beta_d
__device__ __forceinline__ void damp_fric(const DevArgs &a, double mi, double Vi, double Vp,
                                          double Kd, double ex, double ey, double vrx, double vry,
                                          double Fr, double &fx, double &fy) {
    const double vn = vrx * ex + vry * ey;
    const double c = 2.0 * a.rd * sqrt(Kd * mi * Vi * Vp);
    fx = -c * vn * ex;
    fy = -c * vn * ey;
    const double vtx = vrx - vn * ex, vty = vry - vn * ey;
    const double vt = sqrt(vtx * vtx + vty * vty);
    const double vthr = a.mu * Fr * a.dt / mi;
    if (vt > vthr) {  // sliding: mu |F_r| against the tangential relative velocity
        const double g = a.mu * Fr / vt;
        fx -= g * vtx;
        fy -= g * vty;
        count(a, C_SLIP);
    } else {  // sticking: removes the tangential relative velocity in one step
        const double g = mi / a.dt;
        fx -= g * vtx;
        fy -= g * vty;
        count(a, C_STICK);
    }
}

// phi - sin(phi), series below 0.5
__device__ __forceinline__ double phi_minus_sin(double phi) {
    if (phi < 0.5) {
        const double p2 = phi * phi;
        double term = phi * p2 * (1.0 / 6.0), s = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            s += term;
            term *= -p2 / ((2.0 * k + 4.0) * (2.0 * k + 5.0));
        }
        return s;
    }
    return phi - sin(phi);
}

// |S| (Rc - |c - p|) of the circular segment of central angle phi, divided
// by Rc^3: (phi - sin phi)/2 - (2/3) sin^3(phi/2).  Its Taylor series
// (leading term phi^5/160) is summed for phi < 2, where the two terms cancel.
__device__ __forceinline__ double segment_gap(double phi) {
    if (phi < 2.0) {
        const double p2 = phi * phi;
        double pw = p2 * p2 * phi * (1.0 / 120.0);
        double a5 = 0.03125, b5 = 7.59375;  // 0.5^5, 1.5^5
        double h = 0.0;
#pragma unroll
        for (int k = 2; k < 18; ++k) {
            const double ck = -0.5 - 0.5 * a5 + b5 * (1.0 / 6.0);
            h += (k & 1) ? -ck * pw : ck * pw;
            pw *= p2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
            a5 *= 0.25;
            b5 *= 2.25;
        }
        return h;
    }
    const double sh = sin(0.5 * phi);
    return 0.5 * (phi - sin(phi)) - (2.0 / 3.0) * sh * sh * sh;
}

// one wall region of area A acting on node i: repulsion Fr along -e (e from
// the node toward the region's centroid), damping and friction against the
// region's velocity (0, wvy)
__device__ __forceinline__ void wall_region(const DevArgs &a, double Kn, double A, double Fr,
                                            double ex, double ey, double wvy, double vxi,
                                            double vyi, double mi, double Vi, double sign,
                                            double &fx, double &fy) {
    double dfx, dfy;
    damp_fric(a, mi, Vi, A, Kn, ex, ey, vxi, vyi - wvy, fabs(Fr), dfx, dfy);
    fx += sign * (-Fr * ex + dfx);
    fy += sign * (-Fr * ey + dfy);
    count(a, C_WALL);
}

// Walls of node i (Sec. 4.5): lane `part` of the node's quad takes wall
// `part` (left, right, floor, top) and the corner `part` of (left, floor),
// (floor, right), (right, top), (top, left), whose region is subtracted
// (inclusion-exclusion, eq. wall-total).
// The same for one lane's wall and corner, returned apart: seg (the wall
// `part`'s segment region) and cor (the corner `part`, already subtracted).
__device__ void wall_parts(const DevArgs &a, int ag, int part, double px, double py, double vxi,
                           double vyi, double mi, double Vi, double Kn, double t, double &sgx,
                           double &sgy, double &crx, double &cry, int &st);

__device__ void wall_forces(const DevArgs &a, int ag, int part, double px, double py, double vxi,
                            double vyi, double mi, double Vi, double Kn, double t, double &fx,
                            double &fy, int &st) {
    double sgx = 0.0, sgy = 0.0, crx = 0.0, cry = 0.0;
    wall_parts(a, ag, part, px, py, vxi, vyi, mi, Vi, Kn, t, sgx, sgy, crx, cry, st);
    fx += sgx;
    fy += sgy;
    fx += crx;
    fy += cry;
}

// whether node p is within R_c of a wall of its aggregate, or beyond one
// (the same test as the quick exit of wall_parts)
__device__ __forceinline__ bool near_wall(const DevArgs &a, int ag, double px, double py,
                                          double t) {
    const double Rc = a.Rc;
    const double *b = a.box + 4 * ag;
    return !(px - b[0] >= Rc && b[1] - px >= Rc && py - b[2] >= Rc &&
             (b[3] - a.vtop[ag] * t) - py >= Rc);
}

__device__ void wall_parts(const DevArgs &a, int ag, int part, double px, double py, double vxi,
                           double vyi, double mi, double Vi, double Kn, double t, double &fx,
                           double &fy, double &crx, double &cry, int &st) {
    const double Rc = a.Rc;
    const double vtop = a.vtop[ag];
    const double d[4] = {px - a.box[4 * ag], a.box[4 * ag + 1] - px, py - a.box[4 * ag + 2],
                         (a.box[4 * ag + 3] - vtop * t) - py};
    if (!(d[part] > -Rc)) st |= kStEscaped;
    // quick exit: far from every wall
    if (d[0] >= Rc && d[1] >= Rc && d[2] >= Rc && d[3] >= Rc) return;
    const double nx[4] = {-1.0, 1.0, 0.0, 0.0}, ny[4] = {0.0, 0.0, -1.0, 1.0};
    const double wv[4] = {0.0, 0.0, 0.0, -vtop};
    {
        const int w = part;
        if (d[w] < Rc && d[w] > -Rc) {
            // circular segment beyond the wall: area (Rc^2/2)(phi - sin phi),
            // phi = 4 asin(sqrt((Rc - d)/(2 Rc)))
            const double phi = 4.0 * asin(sqrt((Rc - d[w]) / (2.0 * Rc)));
            const double A = 0.5 * Rc * Rc * phi_minus_sin(phi);
            if (A > 0.0) {
                // K_n (Rc - |c - p|) V_i |S| without cancellation as d -> Rc
                const double Fr = Kn * Vi * (Rc * Rc * Rc * segment_gap(phi));
                wall_region(a, Kn, A, Fr, nx[w], ny[w], wv[w], vxi, vyi, mi, Vi, 1.0, fx, fy);
            }
        }
    }
    const int pa[4] = {0, 2, 1, 3}, pb[4] = {2, 1, 3, 0};
    const int wa = pa[part], wb = pb[part];
    const double da = d[wa], db = d[wb];
    // the two segments overlap iff the quadrant beyond both walls comes
    // within Rc of the node (for da, db >= 0: da^2 + db^2 < Rc^2)
    const double qa = da > 0.0 ? da : 0.0, qb = db > 0.0 ? db : 0.0;
    if (!(da > -Rc && db > -Rc && qa * qa + qb * qb < Rc * Rc)) return;
    double A, Ix, Iy;
    if (da * da + db * db < Rc * Rc) {
        // the corner (da, db) inside the disk: triangle (da,db)-(x2,db)-(da,y1)
        // plus the circular segment on its hypotenuse
        const double x2 = sqrt((Rc - db) * (Rc + db)), y1 = sqrt((Rc - da) * (Rc + da));
        const double D = (Rc - da) * (Rc + da) - db * db;
        const double wx = da > 0.0 ? D / (x2 + da) : x2 - da;
        const double wy = db > 0.0 ? D / (y1 + db) : y1 - db;
        const double At = 0.5 * wx * wy;
        const double chord = sqrt(wx * wx + wy * wy);
        const double half = asin(chord / (2.0 * Rc));
        const double As = 0.5 * Rc * Rc * phi_minus_sin(2.0 * half);
        const double sh = sin(half);
        const double ms = (2.0 / 3.0) * Rc * Rc * Rc * sh * sh * sh;
        A = At + As;
        if (!(A > 0.0)) return;
        Ix = At * (da + (da + wx) + da) / 3.0 + ms * (wy / chord);
        Iy = At * (db + db + (db + wy)) / 3.0 + ms * (wx / chord);
    } else if (da < 0.0 && db < 0.0) {
        // node beyond both walls, corner outside the disk: the disk minus the
        // two disjoint caps on the near sides of the walls
        const double pa2 = 4.0 * asin(sqrt((Rc + da) / (2.0 * Rc)));
        const double pb2 = 4.0 * asin(sqrt((Rc + db) / (2.0 * Rc)));
        const double qa2 = (Rc - da) * (Rc + da), qb2 = (Rc - db) * (Rc + db);
        A = Rc * Rc * M_PI - 0.5 * Rc * Rc * (phi_minus_sin(pa2) + phi_minus_sin(pb2));
        Ix = (2.0 / 3.0) * qa2 * sqrt(qa2);
        Iy = (2.0 / 3.0) * qb2 * sqrt(qb2);
    } else {
        // node beyond one wall, whose line misses the other wall's segment:
        // the overlap is that whole segment
        const double dd = da < 0.0 ? db : da;
        const double ph = 4.0 * asin(sqrt((Rc - dd) / (2.0 * Rc)));
        const double q2 = (Rc - dd) * (Rc + dd);
        A = 0.5 * Rc * Rc * phi_minus_sin(ph);
        if (!(A > 0.0)) return;
        const double m = (2.0 / 3.0) * q2 * sqrt(q2);
        Ix = da < 0.0 ? 0.0 : m;
        Iy = da < 0.0 ? m : 0.0;
    }
    const double cx = (Ix * nx[wa] + Iy * nx[wb]) / A, cy = (Ix * ny[wa] + Iy * ny[wb]) / A;
    const double dist = sqrt(cx * cx + cy * cy);
    const double wvy = (wa == 3 || wb == 3) ? -vtop : 0.0;
    const double Fr = Kn * (Rc - dist) * Vi * A;
    wall_region(a, Kn, A, Fr, cx / dist, cy / dist, wvy, vxi, vyi, mi, Vi, -1.0, crx, cry);
}

// bond (i, j) is in the reference set and intact (scan of i's own row)
// is j an intact bond partner of i?  Bond rows are in ascending partner
// order: a binary search of the row.
__device__ __forceinline__ bool bonded_intact(const DevArgs &a, int i, int j) {
    const uint32_t base = a.slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
    const int n = a.rowlen[i];
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int jj = (int)(a.col[base + (uint32_t)mid * kSlice] & kIndexMask);
        if (jj < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo == n) return false;
    const uint32_t e = a.col[base + (uint32_t)lo * kSlice];
    return (int)(e & kIndexMask) == j && (e & kBroken) == 0;
}


// Contact of node i with node j at separation (ddx, ddy) = p_j - p_i,
// r2 = |p_j - p_i|^2 < R_c^2, r2 > 0: repulsion (Sec. 4.1 for other
// particles, Sec. 4.4 for unbonded nodes of the same particle), damping and
// friction.  Accumulates into the self or the inter-particle term.
// The partner's reference position (xj, yj), volume Vj and velocity come in
// loaded; its material's stiffness is read only with several materials.
template <typename R>
__device__ __forceinline__ void contact_pair_d(const DevArgs &a, const MatConst &mc, bool same,
                                               int pj, double xi, double yi, double xj, double yj,
                                               double Vj, double ddx, double ddy, double r2,
                                               double vxi, double vyi, double vxj, double vyj,
                                               double Vi, double mi, R &fsx, R &fsy, R &fnx,
                                               R &fny) {
    const double d = sqrt(r2);
    const double ex = ddx / d, ey = ddy / d;
    double coef, Kd;
    if (!same) {
        const double Ka = mc.Kn, Kb = a.M == 1 ? mc.Kn : a.mat[a.pmat[pj]].Kn;
        const double Kn = (2.0 * Ka * Kb) / (Ka + Kb);  // harmonic mean (Sec. 4.1)
        coef = -Kn * (a.Rc - d);
        Kd = Kn;
        count(a, C_INTER);
    } else {
        const double X = xj - xi, Y = yj - yi;
        const double L = sqrt(X * X + Y * Y);  // reference distance |xi|
        if (L < a.Rc)
            coef = (d < L) ? mc.cw * (d - L) / L : 0.0;
        else
            coef = mc.cw * (d - a.Rc) / a.Rc;
        Kd = mc.Kd_self;
        count(a, C_SELF);
    }
    const double Frx = coef * Vi * Vj * ex, Fry = coef * Vi * Vj * ey;
    const double Fr = fabs(coef) * Vi * Vj;
    double dfx, dfy;
    damp_fric(a, mi, Vi, Vj, Kd, ex, ey, vxi - vxj, vyi - vyj, Fr, dfx, dfy);
    if (same) {
        fsx += (R)(Frx + dfx);
        fsy += (R)(Fry + dfy);
    } else {
        fnx += (R)(Frx + dfx);
        fny += (R)(Fry + dfy);
    }
}

template <typename R>
__device__ __forceinline__ void contact_pair(const DevArgs &a, const MatConst &mc, int i, int j,
                                             bool same, int pj, double xi, double yi, double ddx,
                                             double ddy, double r2, double vxi, double vyi,
                                             double vxj, double vyj, double Vi, double mi,
                                             R &fsx, R &fsy, R &fnx, R &fny) {
    contact_pair_d<R>(a, mc, same, pj, xi, yi, a.x[j], a.y[j], a.vol[j], ddx, ddy, r2, vxi, vyi,
                      vxj, vyj, Vi, mi, fsx, fsy, fnx, fny);
}

// LDS written by some lanes of a wavefront and then read by others of it
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Contact candidate list of every node at its advanced position: nodes of
// the 3 x 3 neighbouring cells (cell side >= list radius) closer than the
// list radius, except intact bonds, in ascending partner index.  Also
// records the displacement at which the list was built.
//
// kBlLanes lanes per node, one wavefront per workgroup.  The three cells of
// a row have consecutive keys, so they are one range of the cell-sorted
// arrays; the lanes take the entries of the three ranges in turn, gather
// the accepted partners in LDS (a wavefront ballot gives each its slot) and
// then write each one at its rank among them.
__global__ __launch_bounds__(64) void k_build_list(DevArgs a) {
    extern __shared__ uint32_t bl_lds[];
    constexpr int kNodes = 64 / kBlLanes;
    const int g = threadIdx.x / kBlLanes, l = threadIdx.x % kBlLanes;
    const int i = blockIdx.x * kNodes + g;
    const bool live = i < a.N;
    const int ic = live ? i : a.N - 1;
    const int maxc = a.maxc;
    uint32_t *L = bl_lds + (size_t)g * maxc;
    double pxi, pyi, uxi, uyi;
    advanced_pos(a, ic, true, pxi, pyi, uxi, uyi);
    const int pi = a.part[ic];
    const int ag = a.pagg[pi];
    int cx, cy;
    cell_of(a, ag, pxi, pyi, cx, cy);
    const int ncx = a.agg_ncx[ag], ncy = a.agg_ncy[ag];
    const uint32_t c0 = a.agg_cell0[ag];
    const int xlo = max(cx - 1, 0), xhi = min(cx + 1, ncx - 1);
    // a node whose row holds every same-particle node within eps and none of
    // whose bonds is broken has an intact bond to a same-particle node j iff
    // j passes the reference-bond test (written as the bond build writes it);
    // other nodes search their row
    const bool by_ref = a.row_full[ic] && !a.node_broken[ic];
    const double xr = a.x[ic], yr = a.y[ic];
    const double thr2 = a.mat[a.pmat[pi]].thr2;
    uint32_t beg[3], cnt[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int yy = cy + r - 1;
        uint32_t b = 0xffffffffu, e = 0u;
        if (live && yy >= 0 && yy < ncy) {
            for (int xx = xlo; xx <= xhi; ++xx) {
                const uint32_t c = c0 + (uint32_t)yy * (uint32_t)ncx + (uint32_t)xx;
                const uint32_t s = a.cell_start[c];
                if (s < (uint32_t)a.N && a.skey[s] == c) {
                    b = min(b, s);
                    e = max(e, a.cell_end[c]);
                }
            }
        }
        beg[r] = b;
        cnt[r] = e > b ? e - b : 0u;
    }
    const int T = (int)(cnt[0] + cnt[1] + cnt[2]);
    const unsigned long long gmask = ((1ull << kBlLanes) - 1ull) << (g * kBlLanes);
    const unsigned long long below = (1ull << (threadIdx.x)) - 1ull;
    int n = 0;
    for (int t0 = 0; __any(t0 < T); t0 += kBlLanes) {
        const int t = t0 + l;
        bool acc = false;
        uint32_t j = 0;
        if (t < T) {
            const uint32_t k = t < (int)cnt[0] ? beg[0] + (uint32_t)t
                               : t < (int)(cnt[0] + cnt[1]) ? beg[1] + (uint32_t)(t - (int)cnt[0])
                                                           : beg[2] + (uint32_t)(t - (int)(cnt[0] + cnt[1]));
            j = (uint32_t)a.perm[k];
            if ((int)j != i) {
                const double ddx = a.spx[k] - pxi, ddy = a.spy[k] - pyi;
                acc = ddx * ddx + ddy * ddy < a.Rl2;
                if (acc && a.spart[k] == pi) {
                    if (by_ref) {
                        const double dx = a.x[j] - xr, dy = a.y[j] - yr;
                        acc = !(dx * dx + dy * dy < thr2);
                    } else {
                        acc = !bonded_intact(a, i, (int)j);
                    }
                }
            }
        }
        const unsigned long long bal = __ballot(acc) & gmask;
        const int pos = n + __popcll(bal & below);
        if (acc && pos < maxc) L[pos] = j;
        n += __popcll(bal);
    }
    wave_lds_sync();
    if (!live) return;
    if (n > maxc) {
        if (l == 0) atomicMax(a.overflow, n);
        n = maxc;
    }
    // ascending partner index: the order contact sums run in does not depend
    // on how the list came about (a rebuild or appends after breaks)
    for (int e = l; e < n; e += kBlLanes) {
        const uint32_t v = L[e];
        int rank = 0;
        for (int m = 0; m < n; ++m) rank += L[m] < v ? 1 : 0;
        a.clist[(size_t)rank * a.N + i] = v;
    }
    if (l == 0) {
        a.clist_n[i] = n;
        a.ubx[i] = (float)uxi;
        a.uby[i] = (float)uyi;
    }
}

__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

// the first stale step before a replay: none, or every step of the replay
// when the candidate lists it follows did not fit their slots
__global__ void k_arm_replay(unsigned long long *inv, const int *overflow) {
    *inv = *overflow ? 0ull : ~0ull;
}

// the start of a round of list-mode steps after `step` completed steps: the
// step base, and either no stale step yet, or (a rebuild ahead of the
// replay) the counters the rebuild fills cleared; k_arm_replay then sets
// the stale step
__global__ void k_round_start(DevArgs a, long long step, int rebuild) {
    *a.step_base = step;
    if (rebuild) {
        *a.overflow = 0;
        if (a.wall_n) *a.wall_n = 0ull;
        if (a.cont_n) *a.cont_n = 0ull;
    } else {
        *a.invalid_step = ~0ull;
    }
}

// ---------------------------------------------------------------------------
// the force kernel
// ---------------------------------------------------------------------------
// The value of lane l ^ X (X = 1 or 2) of the same quad: a DPP quad
// permutation (register to register, no LDS round trip).  Every lane of a
// quad is active wherever these are used (quads leave together).
template <int X>
__device__ __forceinline__ int quad_xor(int v) {
    constexpr int ctrl = X == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
}
template <int X>
__device__ __forceinline__ unsigned quad_xor(unsigned v) {
    return (unsigned)quad_xor<X>((int)v);
}
template <int X>
__device__ __forceinline__ float quad_xor(float v) {
    return __int_as_float(quad_xor<X>(__float_as_int(v)));
}
template <int X>
__device__ __forceinline__ double quad_xor(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = quad_xor<X>((int)(b & 0xffffffffll));
    const int hi = quad_xor<X>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum over the four lanes of a node's quad in a fixed order, (l0 + l1) + (l2 + l3)
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
    v += quad_xor<1>(v);
    v += quad_xor<2>(v);
    return v;
}

// the same over the LPN lanes of a node (LPN = 1, 2 or 4 consecutive lanes;
// quad_xor<1> swaps the lanes of each pair): (l0 + l1) + (l2 + l3)
template <int LPN, typename T>
__device__ __forceinline__ T lanes_sum(T v) {
    if constexpr (LPN >= 2) v += quad_xor<1>(v);
    if constexpr (LPN == 4) v += quad_xor<2>(v);
    return v;
}
template <int LPN>
__device__ __forceinline__ int lanes_or(int v) {
    if constexpr (LPN >= 2) v |= quad_xor<1>(v);
    if constexpr (LPN == 4) v |= quad_xor<2>(v);
    return v;
}
template <int LPN>
__device__ __forceinline__ double lanes_max(double v) {
    if constexpr (LPN >= 2) v = fmax(v, quad_xor<1>(v));
    if constexpr (LPN == 4) v = fmax(v, quad_xor<2>(v));
    return v;
}

// The largest SELL-16 row width among the slices of a wavefront's nodes
// (64 / LPN nodes: one slice at LPN 4, two at 2, four at 1), uniform over
// the wavefront so that the slot loop exits on a scalar branch.
template <int LPN>
__device__ __forceinline__ int wave_row_width(int w) {
    if constexpr (LPN == 4) {
        return __builtin_amdgcn_readfirstlane(w);
    } else if constexpr (LPN == 2) {
        return max(__builtin_amdgcn_readlane(w, 0), __builtin_amdgcn_readlane(w, 32));
    } else {
        return max(max(__builtin_amdgcn_readlane(w, 0), __builtin_amdgcn_readlane(w, 16)),
                   max(__builtin_amdgcn_readlane(w, 32), __builtin_amdgcn_readlane(w, 48)));
    }
}

// The start of node i's SELL-16 row for lane `sub`: slice base, row width and
// the lane's first batch of slot words, loaded early (before the workgroup's
// LDS staging) so that these dependent loads overlap the staging loads.
constexpr int kBatch = 8;
struct SlotHead {
    uint32_t base;
    int W;
    uint32_t ev[kBatch];
};

template <int LPN>
__device__ __forceinline__ void slot_head(const DevArgs &a, int i, int sub, SlotHead &h) {
    const uint32_t sl = (uint32_t)i / kSlice;
    const uint32_t p0 = a.slice_ptr[sl], p1 = a.slice_ptr[sl + 1];
    h.base = p0 + (uint32_t)i % kSlice;
    h.W = (int)((p1 - p0) / kSlice);
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
        const int k = sub + LPN * t;
        h.ev[t] = k < h.W ? a.col[h.base + (uint32_t)k * kSlice] : kBroken;
    }
}

// The exact decision of Sec. 3.1 for bond (i, j): the stretch evaluated in
// IEEE FP64 (correctly rounded square roots and division, no contraction:
// the expression the oracle evaluates, bit for bit).
__device__ __forceinline__ bool exact_break(double X, double Y, double EX, double EY, double DX,
                                         double DY, double s0) {
    const double l0x = __dsqrt_rn(__dadd_rn(__dmul_rn(X, X), __dmul_rn(Y, Y)));
    const double lx = __dsqrt_rn(__dadd_rn(__dmul_rn(DX, DX), __dmul_rn(DY, DY)));
    const double nm = __dadd_rn(__dmul_rn(EX, __dadd_rn(DX, X)), __dmul_rn(EY, __dadd_rn(DY, Y)));
    const double sx = __ddiv_rn(nm, __dmul_rn(l0x, __dadd_rn(lx, l0x)));
    return fabs(sx) > s0;
}

// Bond forces of node i from the slots k = sub, sub + LPN, ... of its
// SELL-16 row (lane `sub` of the node's LPN lanes).  Every slot runs the
// same branch-free arithmetic (padding and broken slots are masked), so
// consecutive slots form independent chains the compiler can interleave.  A
// bond whose approximate stretch comes within 1e-10 (FP64) or 2e-6 (FP32) of
// s0 is re-decided by exact_break.
// STAGED: partner data from the workgroup's LDS window (a separate
// instantiation, so that no load merges LDS and global addresses into one
// generic access).
// slot t < 4 of the break log of node i's lane sub: the partners of bonds
// that lane broke in this step
__device__ __forceinline__ size_t brk_slot(int i, int sub, int t) {
    return (((size_t)i << 2) + (size_t)sub) * 4 + (size_t)t;
}

template <typename R, int MODE, bool STAGED, int LPN>
__device__ __forceinline__ void bond_forces(const DevArgs &a, const MatConst &mc, int i, int sub,
                                            int lo, const double *S, double xi,
                                            double yi, double uxi, double uyi, double Vi, R &fpx,
                                            R &fpy, int &nbrk, double &smx,
                                            const SlotHead &h, bool un) {
    constexpr bool adv = (MODE == M_STEP);
    {
        const uint32_t base = h.base;
        const int Wi = h.W;  // this node's slice
        // the widest slice of the wavefront's nodes: the loop below branches on
        // a scalar; a lane past its own row holds padding words (kBroken)
        const int W = wave_row_width<LPN>(Wi);
        const double s0 = mc.s0, s0m = mc.s0 * (1.0 - 1e-10);
        // per node: c_w V_i and c_w V_i / eps; the bond's c_w V_i V_j w with
        // the conic weight w = 1 - l0/eps is V_j (c_w V_i - l0 c_w V_i / eps),
        // and c_w V_i V_j for the constant micromodulus (cVie = 0)
        const double cVi = mc.cw * Vi;
        const double cVie = mc.conic != 0 ? cVi / mc.eps : 0.0;
        // this lane's slots k = sub + LPN t; their words are fetched in batches
        // of kBatch before any of them is used, so the loads overlap (the
        // first batch comes with the row head)
        constexpr int NB = LPN == 4 ? kBatch : kBatch / 2;
        for (int kb = 0; kb < W; kb += LPN * NB) {
            const int k0 = kb + sub;
            uint32_t ev[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const int k = k0 + LPN * t;
                ev[t] = (kb == 0 && t < kBatch) ? h.ev[t < kBatch ? t : 0]
                                                 : (k < Wi ? a.col[base + (uint32_t)k * kSlice] : kBroken);
            }
            // fully unrolled, so that ev[t] is a register and not a select
            // chain; the wavefront leaves at the row's end
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const int k = k0 + LPN * t;
                if (kb + LPN * t >= W) break;
                const uint32_t e = ev[t];
                const bool valid = (e & kBroken) == 0;
                const int j = valid ? (int)e : i;
                double xj, yj, uxj, uyj, Vj;
                if constexpr (STAGED) {
                    const int q = j - lo;
                    // node q of the window: (x, y), (ux, uy), (V, -) as three
                    // aligned 16-byte LDS reads from one address
                    const double *Sq = S + __umul24((unsigned)q, (unsigned)kWin);
                    const double2 pxy = *reinterpret_cast<const double2 *>(Sq);
                    const double2 puv = *reinterpret_cast<const double2 *>(Sq + 2);
                    xj = pxy.x;
                    yj = pxy.y;
                    uxj = puv.x;
                    uyj = puv.y;
                    Vj = Sq[4];
                } else {
                    double pxj, pyj;
                    if (adv)
                        advanced_pos_un(a, j, un, pxj, pyj, uxj, uyj);
                    else
                        advanced_pos(a, j, false, pxj, pyj, uxj, uyj);
                    xj = a.x[j];
                    yj = a.y[j];
                    Vj = a.vol[j];
                }
                // bond xi, relative displacement eta, current bond xi + eta; the
                // stretch eta.(xi + eta + xi) / (|xi| (|xi + eta| + |xi|)) has no
                // cancellation at small strain, so refined hardware square roots
                // give it to a few ulps
                const double X = xj - xi, Y = yj - yi;
                const double EX = uxj - uxi, EY = uyj - uyi;
                const double DX = X + EX, DY = Y + EY;
                // padding slots (j = i) have X = Y = EX = EY = 0: the floors keep
                // their arithmetic finite and their coefficient is zero, as is
                // that of a broken bond
                bool cand;
                R g, DXr, DYr;
                // (the 1e-200 / 1e-30 added under the squares keeps padding
                // finite and is far below an ulp of any bond's length)
                if constexpr (sizeof(R) == 8) {
                    const double l0s = fma(X, X, fma(Y, Y, 1e-200));
                    const double ls = fma(DX, DX, fma(DY, DY, 1e-200));
                    const double l0 = sqrt_nr(l0s), rl = rsq_nr(ls);
                    const double l = ls * rl;
                    const double num = fma(EX, DX + X, EY * (DY + Y));
                    const double s = num * rcp_nr(l0 * (l + l0));
                    cand = valid && fabs(s) > s0m;
                    if (MODE == M_FORCES && valid) smx = fmax(smx, fabs(s));
                    const double vj = valid ? Vj : 0.0;
                    g = (vj * fma(-l0, cVie, cVi)) * s * rl;
                    DXr = DX;
                    DYr = DY;
                } else {
                    const float Xf = (float)X, Yf = (float)Y, DXf = (float)DX, DYf = (float)DY;
                    const float EXf = (float)EX, EYf = (float)EY;
                    const float l0s = fmaf(Xf, Xf, fmaf(Yf, Yf, 1e-30f));
                    const float ls = fmaf(DXf, DXf, fmaf(DYf, DYf, 1e-30f));
                    const float r0 = __builtin_amdgcn_rsqf(l0s), rl = __builtin_amdgcn_rsqf(ls);
                    const float l0 = l0s * r0, l = ls * rl;
                    const float num = fmaf(EXf, DXf + Xf, EYf * (DYf + Yf));
                    const float s = num * __builtin_amdgcn_rcpf(l0 * (l + l0));
                    cand = valid && fabsf(s) > (float)(s0 - 2e-6);
                    if (MODE == M_FORCES && valid) smx = fmax(smx, (double)fabsf(s));
                    const float vj = valid ? (float)Vj : 0.0f;
                    g = (vj * fmaf(-l0, (float)cVie, (float)cVi)) * s * rl;
                    DXr = DXf;
                    DYr = DYf;
                }
                if (cand && exact_break(X, Y, EX, EY, DX, DY, s0)) {
                    // rare: broken for good (Sec. 3.1)
                    if (MODE != M_FORCES) a.col[base + (uint32_t)k * kSlice] = e | kBroken;
                    // partners for the candidate list, logged in memory
                    // rather than held in registers through the loop
                    if (MODE == M_STEP && nbrk < 4) a.brk_log[brk_slot(i, sub, nbrk)] = (uint32_t)j;
                    ++nbrk;
                    g = 0;
                }
                fpx = fma(g, DXr, fpx);
                fpy = fma(g, DYr, fpy);
            }
        }
    }
}

// Contact forces of node i (lane `sub` of its LPN lanes): with candidate
// lists (LIST), the listed candidates j with j mod LPN = sub; otherwise (LPN
// 4) the nodes of the cells sub, sub + 4, sub + 8 of the 3 x 3
// neighbourhood.  Pairs closer than R_c act; an intact bond replaces contact
// between nodes of one particle.
// SOLO: one thread takes lane `sub`'s share by itself (callers that loop
// over sub on one thread), so the node's lanes are not a quad to exchange
// with: candidates are then taken one by one.
template <typename R, bool LIST, bool adv, int LPN = 4, bool SOLO = false>
__device__ __forceinline__ void contact_forces(const DevArgs &a, const MatConst &mc, int i,
                                               int sub, int pi, int ag, double xi, double yi,
                                               double pxi, double pyi, double vxi, double vyi,
                                               double Vi, double mi, R &fsx, R &fsy, R &fnx,
                                               R &fny, int nc_pre = -1, bool un = false) {
    if (LIST) {
        // Candidates listed at the last rebuild (intact bonds excluded), in
        // ascending j, taken in batches of kCB list entries.  First the
        // node's lanes split a batch by position and test the distances (a
        // lane's kPer candidates loaded together: one memory round trip, not
        // one per candidate); then each pair closer than R_c goes to lane
        // j mod LPN, in ascending j, so a lane's sum depends only on the
        // pairs within R_c, not on which extra candidates the list holds (a
        // superset that depends on when it was built).
        const int nc = nc_pre >= 0 ? nc_pre : a.clist_n[i];
        if constexpr (SOLO) {
            for (int q = 0; q < nc; ++q) {
                const int j = (int)a.clist[(size_t)q * a.N + i];
                if ((j & (LPN - 1)) != sub) continue;
                const double xj = a.x[j], yj = a.y[j];
                const double vxj = a.vx[j], vyj = a.vy[j], Vj = a.vol[j];
                const int pj = a.part[j];
                double pxj, pyj, ux, uy;
                if (adv)
                    advanced_pos_un(a, j, un, pxj, pyj, ux, uy);
                else
                    advanced_pos(a, j, false, pxj, pyj, ux, uy);
                const double ddx = pxj - pxi, ddy = pyj - pyi;
                const double r2 = ddx * ddx + ddy * ddy;
                if (!(r2 < a.Rc2)) continue;
                if (r2 == 0.0) {
                    count(a, C_COINC);
                    continue;
                }
                contact_pair_d<R>(a, mc, pj == pi, pj, xi, yi, xj, yj, Vj, ddx, ddy, r2, vxi,
                                  vyi, vxj, vyj, Vi, mi, fsx, fsy, fnx, fny);
            }
            return;
        }
        constexpr int kPer = 4;
        constexpr int kCB = kPer * LPN;
        static_assert(kCB <= 32, "a batch's mask is one word");
        for (int q0 = 0; q0 < nc; q0 += kCB) {
            int jq[kPer];
#pragma unroll
            for (int m = 0; m < kPer; ++m) {
                const int q = q0 + sub + m * LPN;
                jq[m] = q < nc ? (int)a.clist[(size_t)q * a.N + i] : -1;
            }
            double pxq[kPer], pyq[kPer];
#pragma unroll
            for (int m = 0; m < kPer; ++m) {
                const int j = jq[m] >= 0 ? jq[m] : i;
                double ux, uy;
                if (adv)
                    advanced_pos_un(a, j, un, pxq[m], pyq[m], ux, uy);
                else
                    advanced_pos(a, j, false, pxq[m], pyq[m], ux, uy);
            }
            int hit = 0;
#pragma unroll
            for (int m = 0; m < kPer; ++m) {
                const double ddx = pxq[m] - pxi, ddy = pyq[m] - pyi;
                if (jq[m] >= 0 && ddx * ddx + ddy * ddy < a.Rc2) hit |= 1 << (sub + m * LPN);
            }
            hit = lanes_or<LPN>(hit);  // the node's pairs within R_c in this batch
            while (hit) {
                const int t = __builtin_ctz((unsigned)hit);
                hit &= hit - 1;
                const int j = (int)a.clist[(size_t)(q0 + t) * a.N + i];
                if ((j & (LPN - 1)) != sub) continue;
                const double xj = a.x[j], yj = a.y[j];
                const double vxj = a.vx[j], vyj = a.vy[j], Vj = a.vol[j];
                const int pj = a.part[j];
                double pxj, pyj, ux, uy;
                if (adv)
                    advanced_pos_un(a, j, un, pxj, pyj, ux, uy);
                else
                    advanced_pos(a, j, false, pxj, pyj, ux, uy);
                const double ddx = pxj - pxi, ddy = pyj - pyi;
                const double r2 = ddx * ddx + ddy * ddy;
                if (!(r2 < a.Rc2)) continue;  // (the same test as the mask's)
                if (r2 == 0.0) {
                    count(a, C_COINC);
                    continue;
                }
                contact_pair_d<R>(a, mc, pj == pi, pj, xi, yi, xj, yj, Vj, ddx, ddy, r2, vxi, vyi,
                                  vxj, vyj, Vi, mi, fsx, fsy, fnx, fny);
            }
        }
    } else {
        static_assert(LIST || LPN == 4, "the cell search runs with four lanes per node");
        // nodes of the 3 x 3 neighbouring cells, cells sub, sub + 4, sub + 8
        int cx, cy;
        cell_of(a, ag, pxi, pyi, cx, cy);
        const int ncx = a.agg_ncx[ag], ncy = a.agg_ncy[ag];
        const uint32_t c0 = a.agg_cell0[ag];
        for (int c9 = sub; c9 < 9; c9 += 4) {
            const int yy = cy + c9 / 3 - 1, xx = cx + c9 % 3 - 1;
            if (yy < 0 || yy >= ncy || xx < 0 || xx >= ncx) continue;
            const uint32_t c = c0 + (uint32_t)yy * (uint32_t)ncx + (uint32_t)xx;
            const uint32_t s = a.cell_start[c];
            if (s >= (uint32_t)a.N || a.skey[s] != c) continue;
            for (uint32_t k = s; k < (uint32_t)a.N && a.skey[k] == c; ++k) {
                const int j = a.perm[k];
                if (j == i) continue;
                const double ddx = a.spx[k] - pxi, ddy = a.spy[k] - pyi;
                const double r2 = ddx * ddx + ddy * ddy;
                if (!(r2 < a.Rc2)) continue;
                if (r2 == 0.0) {
                    count(a, C_COINC);
                    continue;
                }
                const int pj = a.spart[k];
                const bool same = (pj == pi);
                if (same && bonded_intact(a, i, j)) continue;  // the bond acts
                contact_pair<R>(a, mc, i, j, same, pj, xi, yi, ddx, ddy, r2, vxi, vyi, a.vx[j],
                                a.vy[j], Vi, mi, fsx, fsy, fnx, fny);
            }
        }
    }
}

// LPN lanes per node (1, 2 or 4): lane `sub` of node i takes the bond slots
// k = sub, sub + LPN, ... of the node's SELL-16 row, every LPN-th contact
// candidate and the walls and corners sub, sub + LPN, ...; the node's lanes
// then combine their partial sums in a fixed order and lane 0 integrates.
// Four lanes keep the chain of dependent work per wavefront short (small
// problems, where latency bounds a launch); one lane does the per-node work
// (walls, candidates, reductions, integration) once instead of four times
// (large problems, bound by instruction issue).  LDS holds the block's window
// of bond partners (reference and current positions, volumes).
// The step (or force evaluation) of the nodes of force workgroup `blk`.
// SEL (step mode with the modal closure on): 0 every node; 1 only the nodes
// of particles under the plain bond force (closure nodes are left to
// k_cl_contact and the closure kernels).
template <typename R, int MODE, bool LIST, int SEL, int LPN, bool WP>
__device__ __forceinline__ void force_block(const DevArgs &a, int lds_cap, int blk,
                                            long long sprev, double *lds) {
    static_assert(LPN == 1 || LPN == 2 || LPN == 4, "1, 2 or 4 lanes per node");
    double *S = lds;  // the window, kWin doubles per node
    constexpr bool adv = (MODE == M_STEP);
    const int sub = threadIdx.x & (LPN - 1);
    const int i = blk * (blockDim.x / LPN) + (threadIdx.x / LPN);
    if (SEL == 1) {
        const int mine = (i < a.N && !a.cl_on[a.part[i]]) ? 1 : 0;
        if (!__syncthreads_or(mine)) return;
    }
    // this node's own data and the head of its bond row, issued before the
    // staging loads (indices clamped: the loads of i >= N are discarded)
    const int ic = i < a.N ? i : a.N - 1;
    const double xi = a.x[ic], yi = a.y[ic];
    // list-mode steps after the first of a replay (closure off) read the
    // advanced displacements the previous launch wrote (uniform over the grid)
    const bool un = LIST && adv && SEL == 0 && a.chunk_k > 0 && a.unx && !a.cl_on;
    double pxi, pyi, uxi, uyi;
    if (adv)
        advanced_pos_un(a, ic, un, pxi, pyi, uxi, uyi);
    else
        advanced_pos(a, ic, false, pxi, pyi, uxi, uyi);
    const double vxi = a.vx[ic], vyi = a.vy[ic];  // velocities of the previous step
    const double Vi = a.vol[ic];
    const int pi = a.part[ic];
    SlotHead head;
    slot_head<LPN>(a, ic, sub, head);
    const int nc_pre = LIST ? a.clist_n[ic] : -1;
    // the epilogue's own-node loads: with four lanes, issued now rather than
    // at the end (the launch is latency-bound); with fewer, at the end (the
    // registers they would hold through the bond loop are scarcer there)
    double axi = 0.0, ayi = 0.0, ubxi = 0.0, ubyi = 0.0;
    if constexpr (LPN == 4) {
        axi = a.ax[ic];
        ayi = a.ay[ic];
        ubxi = LIST ? (double)a.ubx[ic] : 0.0;
        ubyi = LIST ? (double)a.uby[ic] : 0.0;
    }
    int lo = 0;
    bool staged = false;
    if (SEL == 0 && a.use_lds) {
        lo = a.win_lo[blk];
        const int cnt = a.win_hi[blk] - lo + 1;
        staged = cnt > 0 && cnt <= lds_cap;
        if (staged) {
            for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
                const int j = lo + k;
                double px, py, ux, uy;
                if (adv)
                    advanced_pos_un(a, j, un, px, py, ux, uy);
                else
                    advanced_pos(a, j, false, px, py, ux, uy);
                *reinterpret_cast<double2 *>(S + kWin * k) = make_double2(a.x[j], a.y[j]);
                *reinterpret_cast<double2 *>(S + kWin * k + 2) = make_double2(ux, uy);
                S[kWin * k + 4] = a.vol[j];
            }
        }
        __syncthreads();
    }
    if (i >= a.N) return;  // a node's lanes leave together

    const int mt = a.pmat[pi];
    const int ag = a.pagg[pi];
    const MatConst mc = a.mat[mt];
    const double mi = mc.rho * Vi;  // the nodal mass, as the host computes it
    // wall time of this evaluation
    const double t = LIST ? (double)(sprev + 1) * a.dt : (double)(*a.step) * a.dt;
    int st = 0;

    R fsx = 0, fsy = 0, fnx = 0, fny = 0, fpx = 0, fpy = 0;
    double fwx = 0.0, fwy = 0.0;
    int nbrk = 0;
    double smx = 0.0;
    // a particle under the modal closure: no bond forces here; its external
    // nodal force goes to the closure kernels, which integrate its nodes
    const bool closure = MODE == M_STEP && a.cl_on && a.cl_on[pi];
    if (SEL == 1 && closure) return;   // a node's lanes leave together
    // List mode runs the bond loop first (its contact candidates never
    // involve intact bonds, so the order does not matter there), which keeps
    // fewer partial sums live through the loop.  Otherwise contact comes
    // first, because self-contact needs the bonds intact at the start of the
    // step and the bond loop commits breaks.
    // (list mode: the walls come after the lanes' sums and the list appends
    // below, where fewer values are live)
    if constexpr (LIST) {
        if (!closure)
            staged ? bond_forces<R, MODE, true, LPN>(a, mc, i, sub, lo, S, xi, yi, uxi,
                                                     uyi, Vi, fpx, fpy, nbrk, smx, head, un)
                   : bond_forces<R, MODE, false, LPN>(a, mc, i, sub, lo, S, xi, yi, uxi,
                                                      uyi, Vi, fpx, fpy, nbrk, smx, head, un);
        // (with the pass, the candidates were evaluated before this launch)
        if constexpr (!WP)
            contact_forces<R, LIST, adv, LPN>(a, mc, i, sub, pi, ag, xi, yi, pxi, pyi, vxi, vyi,
                                              Vi, mi, fsx, fsy, fnx, fny, nc_pre, un);
    } else {
        contact_forces<R, LIST, adv, LPN>(a, mc, i, sub, pi, ag, xi, yi, pxi, pyi, vxi, vyi, Vi,
                                          mi, fsx, fsy, fnx, fny);
#pragma unroll 1
        for (int part = sub; part < 4; part += LPN)
            wall_forces(a, ag, part, pxi, pyi, vxi, vyi, mi, Vi, mc.Kn, t, fwx, fwy, st);
        if (!closure)
            staged ? bond_forces<R, MODE, true, LPN>(a, mc, i, sub, lo, S, xi, yi, uxi,
                                                     uyi, Vi, fpx, fpy, nbrk, smx, head, false)
                   : bond_forces<R, MODE, false, LPN>(a, mc, i, sub, lo, S, xi, yi, uxi,
                                                      uyi, Vi, fpx, fpy, nbrk, smx, head, false);
    }

    // a lane that broke one of the node's bonds marks the node (the list
    // build then searches its row)
    if (MODE != M_FORCES && nbrk > 0) a.node_broken[i] = 1;

    // ---- combine the node's lanes -----------------------------------------------
    fpx = lanes_sum<LPN>(fpx);
    fpy = lanes_sum<LPN>(fpy);
    fsx = lanes_sum<LPN>(fsx);
    fsy = lanes_sum<LPN>(fsy);
    fnx = lanes_sum<LPN>(fnx);
    fny = lanes_sum<LPN>(fny);
    if constexpr (LIST && WP) {
        // the pass's sums over this node's candidates (its lanes, its order)
        if (sub == 0 && nc_pre > 0) {
            const double2 c0 = *reinterpret_cast<const double2 *>(a.csum + 4 * (size_t)i);
            const double2 c1 = *reinterpret_cast<const double2 *>(a.csum + 4 * (size_t)i + 2);
            fsx = (R)c0.x;
            fsy = (R)c0.y;
            fnx = (R)c1.x;
            fny = (R)c1.y;
        }
    }
    if constexpr (LPN != 4) {
        axi = a.ax[i];
        ayi = a.ay[i];
        ubxi = LIST ? (double)a.ubx[i] : 0.0;
        ubyi = LIST ? (double)a.uby[i] : 0.0;
    }
    // list mode: a bond that broke makes its pair a self-contact candidate
    // from the next step on; if the pair was within the list radius at the
    // last rebuild (build-time positions, with a margin), this lane appends it
    // to the node's own candidate list, in lane order; a full list means a
    // rebuild instead
    bool relist = false;
    // (skipped by a wavefront without a break: none of its nodes has anything to append)
    if (LIST && MODE == M_STEP && __any(nbrk > 0)) {
        int keep = 0;
        uint32_t kj[4];
        const int nb = nbrk < 4 ? nbrk : 4;
        if (nb) {
            const double bxi = xi + ubxi, byi = yi + ubyi;
            for (int t = 0; t < nb; ++t) {
                const int j = (int)a.brk_log[brk_slot(i, sub, t)];
                const double dx = (a.x[j] + (double)a.ubx[j]) - bxi;
                const double dy = (a.y[j] + (double)a.uby[j]) - byi;
                if (dx * dx + dy * dy < a.Rl2 * (1.0 + 1e-6)) kj[keep++] = (uint32_t)j;
            }
        }
        for (int t = keep; t < 4; ++t) kj[t] = 0xffffffffu;
        const int over = lanes_or<LPN>(nbrk > 4 ? 1 : 0);
        const int tot = lanes_sum<LPN>(keep);
        // lane 0 gathers the partners of the node's lanes and merges them into
        // the node's sorted list
        uint32_t nj[4 * LPN];
        const int q0 = (int)(threadIdx.x & ~(unsigned)(LPN - 1));
#pragma unroll
        for (int l = 0; l < LPN; ++l)
#pragma unroll
            for (int t = 0; t < 4; ++t) nj[4 * l + t] = __shfl(kj[t], q0 + l, 64);
        if (over || nc_pre + tot > a.maxc) {
            relist = true;
        } else if (sub == 0 && tot) {
            int n = nc_pre;
            for (int e = 0; e < 4 * LPN; ++e) {
                const uint32_t v = nj[e];
                if (v == 0xffffffffu) continue;
                int m = n - 1;
                while (m >= 0 && a.clist[(size_t)m * a.N + i] > v) {
                    a.clist[(size_t)(m + 1) * a.N + i] = a.clist[(size_t)m * a.N + i];
                    --m;
                }
                a.clist[(size_t)(m + 1) * a.N + i] = v;
                ++n;
            }
            a.clist_n[i] = n;
            // with the pass: a node's first candidates put it on its list
            if (WP && nc_pre == 0) a.cont_list[atomicAdd(a.cont_n, 1ull)] = i;
        }
    }
    if constexpr (LIST && WP) {
        // the pass evaluated this node's wall force before this launch
        // (every node near a wall is on its list until the next rebuild)
        if (sub == 0 && __builtin_expect(near_wall(a, ag, pxi, pyi, t), 0)) {
            fwx = a.wfx[i];
            fwy = a.wfy[i];
        }
    } else if constexpr (LIST) {
        // (most nodes are far from every wall: the loop is the cold path)
        if (__builtin_expect(near_wall(a, ag, pxi, pyi, t), 0)) {
#pragma unroll
            for (int part = sub; part < 4; part += LPN)
                wall_forces(a, ag, part, pxi, pyi, vxi, vyi, mi, Vi, mc.Kn, t, fwx, fwy, st);
        }
    }
    fwx = lanes_sum<LPN>(fwx);
    fwy = lanes_sum<LPN>(fwy);
    nbrk = lanes_sum<LPN>(nbrk);
    st = lanes_or<LPN>(st);
    if (MODE == M_FORCES) smx = lanes_max<LPN>(smx);
    if (sub != 0) return;
    if (MODE != M_FORCES) count(a, C_BROKEN, (unsigned long long)nbrk);
    if (LIST && relist) atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));

    // ---- outputs ---------------------------------------------------------------
    const double Fx = (((double)fpx + (double)fsx) + (double)fnx) + fwx;
    const double Fy = (((double)fpy + (double)fsy) + (double)fny) + fwy;
    if (MODE == M_FORCES) {
        const int N = a.N;
        double *T = a.terms;
        T[0 * N + i] = (double)fpx / Vi;
        T[1 * N + i] = (double)fpy / Vi;
        T[2 * N + i] = (double)fsx / Vi;
        T[3 * N + i] = (double)fsy / Vi;
        T[4 * N + i] = (double)fnx / Vi;
        T[5 * N + i] = (double)fny / Vi;
        T[6 * N + i] = fwx / Vi;
        T[7 * N + i] = fwy / Vi;
        T[8 * N + i] = mi * a.gx / Vi;
        T[9 * N + i] = mi * a.gy / Vi;
        if (a.smax) a.smax[i] = smx;
    } else if (closure) {
        a.cl_fx[i] = ((double)fsx + (double)fnx) + fwx;
        a.cl_fy[i] = ((double)fsy + (double)fny) + fwy;
        a.ux_o[i] = uxi;
        a.uy_o[i] = uyi;
        if (!(isfinite(uxi) && isfinite(uyi))) st |= kStNonfinite;
    } else {
        const double axn = Fx / mi + a.gx, ayn = Fy / mi + a.gy;
        a.ax_o[i] = axn;
        a.ay_o[i] = ayn;
        if (MODE == M_STEP) {
            const double vxn = vxi + a.hdt * (axi + axn);
            const double vyn = vyi + a.hdt * (ayi + ayn);
            a.vx_o[i] = vxn;
            a.vy_o[i] = vyn;
            a.ux_o[i] = uxi;
            a.uy_o[i] = uyi;
            if (!(isfinite(uxi) && isfinite(uyi) && isfinite(vxn) && isfinite(vyn)))
                st |= kStNonfinite;
            if (LIST) {
                // the next step's displacement against the one the list was built at
                const double unx = (uxi + a.dt * vxn) + a.hdt2 * axn;
                const double uny = (uyi + a.dt * vyn) + a.hdt2 * ayn;
                if (a.unx_o) {  // for the next launch of the replay
                    a.unx_o[i] = unx;
                    a.uny_o[i] = uny;
                }
                const double ex = unx - ubxi, ey = uny - ubyi;
                if (!(ex * ex + ey * ey <= a.move2))
                    atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));
            }
        }
    }
    if (st) atomicOr(a.status, st);
}

// Workgroups are dispatched to the eight XCDs in turn (workgroup w to XCD
// w mod 8), each XCD with its own L2.  Map them so that each XCD takes one
// contiguous range of node blocks: neighbouring blocks share most of their
// partner windows and contact partners, which then meet in the same L2.
__device__ __forceinline__ int xcd_block(int w, int nb) {
    constexpr int kXcd = 8;
    const int x = w % kXcd, r = w / kXcd;
    const int q = nb / kXcd, rem = nb % kXcd;
    return x * q + min(x, rem) + r;  // a bijection of [0, nb)
}

template <typename R, int MODE, bool LIST, int SEL = 0, int LPN = 4>
__global__ __launch_bounds__(1024) void k_force(DevArgs a, int lds_cap) {
    extern __shared__ double lds[];
    // list mode: this launch computes step sprev + 1 of a replay that started
    // after step *step_base; once a list has gone stale, that step and every
    // later one of the replay are no-ops (the check is uniform over the grid)
    long long sprev = 0;
    if (LIST) {
        sprev = *a.step_base + a.chunk_k;
        if ((unsigned long long)(sprev + 1) >= *a.invalid_step) return;
    }
    if (SEL == 1) {
        // slots blockIdx.x, + gridDim.x, ... of the list of force workgroups
        // that hold nodes under the plain force (listed at switch-on, appended
        // by the kernels that make a particle fall back from the closure); no
        // LDS staging.  The list cannot grow during this launch.
        const int nl = *a.n_pd_blocks;
        for (int slot = blockIdx.x; slot < nl; slot += gridDim.x)
            force_block<R, MODE, LIST, SEL, LPN, false>(a, 0, a.pd_blocks[slot], sprev, lds);
    } else {
        force_block<R, MODE, LIST, SEL, LPN, false>(a, lds_cap, xcd_block(blockIdx.x, gridDim.x),
                                                    sprev, lds);
    }
}

// the list-mode step with the pass of walls and contact candidates: without
// their code the kernel fits in 80 VGPRs at one or two lanes per node (six
// wavefronts per SIMD instead of four) and in 96 at four (five)
template <typename R, int LPN>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(LPN == 4 ? 5 : 6, 8))) void k_force_wp(
    DevArgs a, int lds_cap) {
    extern __shared__ double lds[];
    const long long sprev = *a.step_base + a.chunk_k;
    if ((unsigned long long)(sprev + 1) >= *a.invalid_step) return;
    force_block<R, M_STEP, true, 0, LPN, true>(a, lds_cap, xcd_block(blockIdx.x, gridDim.x), sprev,
                                               lds);
}

// Contact and wall forces of a node of a particle under the modal closure
// (list mode): every candidate and every wall and corner region in turn.
// The closure kernels integrate these nodes.
struct ClNode {
    double fx, fy, ux, uy;  // external force, advanced displacement
};

template <typename R>
__device__ __forceinline__ ClNode cl_contact_node(const DevArgs &a, int i, long long sprev) {
    const int pi = a.part[i];
    const double xi = a.x[i], yi = a.y[i];
    double pxi, pyi, uxi, uyi;
    advanced_pos(a, i, true, pxi, pyi, uxi, uyi);
    const double vxi = a.vx[i], vyi = a.vy[i];
    const double Vi = a.vol[i], mi = a.mass[i];
    const int ag = a.pagg[pi];
    const MatConst mc = a.mat[a.pmat[pi]];
    const double t = (double)(sprev + 1) * a.dt;
    int st = 0;
    R fsx = 0, fsy = 0, fnx = 0, fny = 0;
    double fwx = 0.0, fwy = 0.0;
#pragma unroll 1
    for (int sub = 0; sub < 4; ++sub)
        contact_forces<R, true, true, 4, true>(a, mc, i, sub, pi, ag, xi, yi, pxi, pyi, vxi, vyi,
                                               Vi, mi, fsx, fsy, fnx, fny);
#pragma unroll 1
    for (int part = 0; part < 4; ++part)
        wall_forces(a, ag, part, pxi, pyi, vxi, vyi, mi, Vi, mc.Kn, t, fwx, fwy, st);
    const double fx = ((double)fsx + (double)fnx) + fwx;
    const double fy = ((double)fsy + (double)fny) + fwy;
    a.cl_fx[i] = fx;
    a.cl_fy[i] = fy;
    a.ux_o[i] = uxi;
    a.uy_o[i] = uyi;
    if (!(isfinite(uxi) && isfinite(uyi))) st |= kStNonfinite;
    if (st) atomicOr(a.status, st);
    return ClNode{fx, fy, uxi, uyi};
}

// every node of the closure particles, a thread per node
template <typename R>
__global__ __launch_bounds__(256) void k_cl_contact(DevArgs a) {
    const long long sprev = *a.step_base + a.chunk_k;
    if ((unsigned long long)(sprev + 1) >= *a.invalid_step) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N || !a.cl_on[a.part[i]]) return;
    cl_contact_node<R>(a, i, sprev);
}

// ---------------------------------------------------------------------------
// the step of the reduced closure in one launch: one workgroup per block of
// at most 16 closure particles of one shape (the MLP's row block) and NW
// wavefronts, each taking the block's particles wv, wv + NW, ...  Per
// particle, on its wavefront: the reduced positions advanced, the contact and
// wall forces of its active nodes and their total force, torque about the
// centroid, contact load and modal force (nodes lane, lane + 64, ... of the
// active list on each lane, summed by butterflies: a fixed order).  Then, for
// the learned closure, the MLP on the block's 16 rows of modal amplitudes,
// all NW wavefronts on the matrix cores (rows of particles that are off or
// past the block are zero).  Then per particle the rates, the gate, the
// reconstruction of the active nodes (every node of a particle that leaves
// the closure) and the motion bound since the last list rebuild.  What a
// particle's first part leaves for its last (modal amplitudes and forces,
// the advanced centroid and angle, the sums) stays in LDS.
// ---------------------------------------------------------------------------
constexpr int kRcWaves = 8;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}


enum { RW_CX = 0, RW_CY, RW_PH, RW_FX, RW_FY, RW_TAU, RW_CONTACT, RW_STRAIN, RW_BQ, RW_N };

template <typename R, bool LEARNED, int NW>
__global__ __launch_bounds__(64 * NW) void k_rc_fused(DevArgs a, ClArgs c, MlpArgs m, int list) {
    __shared__ __align__(16) uint16_t Xs[16 * kXsStride];
    __shared__ __align__(16) uint16_t H1[LEARNED ? 16 * kHStride : 8];
    __shared__ __align__(16) uint16_t H2[LEARNED ? 16 * kHStride : 8];
    __shared__ double Gh[LEARNED ? 16 : 1][kClModes];
    __shared__ double Ge[16][kClModes];
    __shared__ double Qs[16][3][kClModes];
    __shared__ double Rw[16][RW_N];
    __shared__ double FB[NW][2][64];
    if (replay_stale(a, list != 0)) return;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rb = blockIdx.x;
    const int s = c.rb_shape[rb], first = c.rb_first[rb], cnt = c.rb_count[rb];
    const long long sprev = *a.step_base + a.chunk_k;
    const int t0 = c.toff[s];
    const int k = l & 31;  // this lane's mode (lanes k and k + 32 hold the same one)
    // ---- per particle: advance, contact, sums ------------------------------------
#pragma unroll 1
    for (int row = wv; row < 16; row += NW) {
        const int ci = first + min(row, cnt - 1);
        const int p = c.cpart[ci];
        const bool on = row < cnt && a.cl_on[p] != 0;  // the same on every lane of the wave
        if (!on) {
            if (LEARNED && l < kClModes) Xs[row * kXsStride + k] = 0;
            continue;
        }
        const int n0 = c.poff[p];
        const int *al = c.alist + (size_t)ci * c.max_n;
        double *RS = c.rs + (size_t)ci * 16;
        const size_t qk = (size_t)ci * kClModes + k;
        const double q = (c.qr[qk] + a.dt * c.qv[qk]) + a.hdt2 * c.qa[qk];
        const double cx = (RS[RS_CX] + a.dt * RS[RS_VX]) + a.hdt2 * RS[RS_AX];
        const double cy = (RS[RS_CY] + a.dt * RS[RS_VY]) + a.hdt2 * RS[RS_AY];
        const double ph = (RS[RS_PHI] + a.dt * RS[RS_OM]) + a.hdt2 * RS[RS_AL];
        if (l < kClModes) {
            c.qr[qk] = q;
            c.q[qk] = q;
            Qs[row][0][k] = q;
        }
        if (l == 0) {
            RS[RS_CX] = cx;
            RS[RS_CY] = cy;
            RS[RS_PHI] = ph;
        }
        const double cp = cos(ph), sp = sin(ph);
        // contact and walls of the active nodes, and their sums
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0, g = 0.0;
        const int na = c.acnt[ci];
        for (int b0 = 0; b0 < na; b0 += 64) {
            const int b = b0 + l;
            double fbx = 0.0, fby = 0.0;
            if (b < na) {
                const int i = al[b];
                const ClNode f = cl_contact_node<R>(a, i, sprev);
                const double Yx = (a.x[i] + f.ux) - cx, Yy = (a.y[i] + f.uy) - cy;
                v0 += f.fx;
                v1 += f.fy;
                v2 += Yx * f.fy - Yy * f.fx;
                v3 += sqrt(f.fx * f.fx + f.fy * f.fy);
                fbx = cp * f.fx + sp * f.fy;  // in the body frame
                fby = -sp * f.fx + cp * f.fy;
            }
            FB[wv][0][l] = fbx;
            FB[wv][1][l] = fby;
            wave_lds_sync();
            // modal force: lane k + 32 h takes the chunk's nodes h, h + 2, ...
            const int nb = min(64, na - b0);
            for (int u = l >> 5; u < nb; u += 2) {
                const int t = t0 + (al[b0 + u] - n0);
                const float px = c.phi[((size_t)t * kClModes + k) * 2];
                const float py = c.phi[((size_t)t * kClModes + k) * 2 + 1];
                g += (double)px * FB[wv][0][u] + (double)py * FB[wv][1][u];
            }
            wave_lds_sync();
        }
        v0 = wave_sum(v0);
        v1 = wave_sum(v1);
        v2 = wave_sum(v2);
        v3 = wave_sum(v3);
        const double ge = g + __shfl_xor(g, 32, 64);
        double sb = fabs(q) * c.sig[s * kClModes + k];
        double bq = 2.0 * c.bvec[s * kClModes + k] * q + q * q;
        for (int o = 16; o > 0; o >>= 1) {  // over the 32 modes
            sb += __shfl_xor(sb, o, 64);
            bq += __shfl_xor(bq, o, 64);
        }
        if (l < kClModes) {
            c.gext[qk] = ge;
            Ge[row][k] = ge;
            if (LEARNED)
                Xs[row * kXsStride + k] = f2bf((float)(q / (double)m.sig_q[s * kClModes + k]));
        }
        if (l == 0) {
            Rw[row][RW_CX] = cx;
            Rw[row][RW_CY] = cy;
            Rw[row][RW_PH] = ph;
            Rw[row][RW_FX] = v0;
            Rw[row][RW_FY] = v1;
            Rw[row][RW_TAU] = v2;
            Rw[row][RW_CONTACT] = v3;
            Rw[row][RW_STRAIN] = sb;
            Rw[row][RW_BQ] = bq;
        }
    }
    // ---- the MLP on the block's rows ----------------------------------------------
    if constexpr (LEARNED) {
        MlpWave<NW> W;
        mlp_load<NW>(W, m.wfr + (size_t)s * kClFrag, m.wf + (size_t)s * kClParams, wv, l);
        __syncthreads();
        mlp_hidden(Xs, kXsStride, W.w1, W.b1, H1, wv, l, 0, 0, nullptr, nullptr);
        __syncthreads();
        mlp_hidden(H1, kHStride, W.w2, W.b2, H2, wv, l, 0, 0, nullptr, nullptr);
        __syncthreads();
        if (wv < kClModes / 16) {
            const f32x4 y = mlp_out<NW>(H2, W, l);
            const int n3 = 16 * wv + (l & 15), kq = 4 * (l >> 4);
            const double lam3 = m.lam[s * kClModes + n3];
            const double sr3 = (double)m.sig_r[s * kClModes + n3];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = kq + t;
                if (row < cnt) Gh[row][n3] = -lam3 * Qs[row][0][n3] + sr3 * (double)y[t];
            }
        }
    }
    __syncthreads();
    // ---- per particle: rates, gate, reconstruction, motion bound -------------------
#pragma unroll 1
    for (int row = wv; row < cnt; row += NW) {
        const int ci = first + row;
        const int p = c.cpart[ci];
        if (a.cl_on[p] == 0) continue;  // off before this step (nothing above changes it)
        const int n0 = c.poff[p];
        const int *al = c.alist + (size_t)ci * c.max_n;
        double *RS = c.rs + (size_t)ci * 16;
        const size_t qk = (size_t)ci * kClModes + k;
        const double q = Qs[row][0][k];
        const double gk = LEARNED ? Gh[row][k] : -c.lam[s * kClModes + k] * q;
        const double qa = gk + Ge[row][k];
        const double qv = c.qv[qk] + a.hdt * (c.qa[qk] + qa);
        if (l < kClModes) {
            c.qv[qk] = qv;
            c.qa[qk] = qa;
            Qs[row][1][k] = qv;
            Qs[row][2][k] = qa;
        }
        const double pm = c.phimax[s * kClModes + k];
        const double qb = c.qrb[qk];
        double dq = fabs(((q + a.dt * qv) + a.hdt2 * qa) - qb) * pm;
        double zq = fabs(qb) * pm;
        for (int o = 16; o > 0; o >>= 1) {
            dq += __shfl_xor(dq, o, 64);
            zq += __shfl_xor(zq, o, 64);
        }
        const double cx = Rw[row][RW_CX], cy = Rw[row][RW_CY], ph = Rw[row][RW_PH];
        const double M = c.Mt[s];
        const double ax = Rw[row][RW_FX] / M + a.gx, ay = Rw[row][RW_FY] / M + a.gy;
        const double alp = Rw[row][RW_TAU] / (c.I0[s] + Rw[row][RW_BQ]);
        const double vx = RS[RS_VX] + a.hdt * (RS[RS_AX] + ax);
        const double vy = RS[RS_VY] + a.hdt * (RS[RS_AY] + ay);
        const double om = RS[RS_OM] + a.hdt * (RS[RS_AL] + alp);
        const double rbx = RS[RS_RBX], rby = RS[RS_RBY], rbphi = RS[RS_RBPHI];
        // the gate for the next step: past gate_frac s0 on the stretch bound or
        // past tau_c on the contact load, the particle leaves the closure with
        // every node reconstructed now
        const bool off = Rw[row][RW_STRAIN] > c.gate_frac * c.s0[s] ||
                         Rw[row][RW_CONTACT] > c.tau_c[s];
        wave_lds_sync();  // Qs complete; every lane has read a.cl_on[p]
        if (l == 0) {
            RS[RS_VX] = vx;
            RS[RS_VY] = vy;
            RS[RS_AX] = ax;
            RS[RS_AY] = ay;
            RS[RS_OM] = om;
            RS[RS_AL] = alp;
            if (off) {
                a.cl_on[p] = 0;
                list_particle_blocks(a, c, p);
                atomicAdd(c.fallbacks, 1ull);
            }
        }
        RcRigid r;
        r.cx = cx;
        r.cy = cy;
        r.vx = vx;
        r.vy = vy;
        r.ax = ax;
        r.ay = ay;
        r.cp = cos(ph);
        r.sp = sin(ph);
        r.om = om;
        r.al = alp;
        const int cntn = off ? c.poff[p + 1] - n0 : c.acnt[ci];
        int st = 0, stale = 0;
        for (int b = l; b < cntn; b += 64) {
            const int i = off ? n0 + b : al[b];
            st |= rc_write(a, c, i, t0 + (i - n0), r, Qs[row][0], Qs[row][1], Qs[row][2], a.ux_o,
                           a.uy_o, a.vx_o, a.vy_o, a.ax_o, a.ay_o);
            if (list && off) {  // a particle leaving the closure: its nodes' own check
                const double unx = (a.ux_o[i] + a.dt * a.vx_o[i]) + a.hdt2 * a.ax_o[i];
                const double uny = (a.uy_o[i] + a.dt * a.vy_o[i]) + a.hdt2 * a.ay_o[i];
                const double ex = unx - (double)a.ubx[i], ey = uny - (double)a.uby[i];
                if (!(ex * ex + ey * ey <= a.move2)) stale = 1;
            }
        }
        if (list && !off) {
            // |c' - c_rb| + |phi' - phi_rb| (r_max + sum |q_rb| phimax) + sum |q' - q_rb| phimax
            // bounds every node's displacement since the rebuild, at the next step
            const double cxn = (cx + a.dt * vx) + a.hdt2 * ax;
            const double cyn = (cy + a.dt * vy) + a.hdt2 * ay;
            const double phn = (ph + a.dt * om) + a.hdt2 * alp;
            const double B = hypot(cxn - rbx, cyn - rby) + fabs(phn - rbphi) * (c.rmax[s] + zq) + dq;
            if (!(B * B <= a.move2)) stale = 1;
        }
        if (st) atomicOr(a.status, st);
        if (__any(stale) && l == 0) atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));
    }
}

hipError_t launch_cl_contact(const DevArgs &a, int precision, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    if (!(a.cl_on && a.cl_fx && a.cl_fy)) return hipErrorInvalidValue;
    const dim3 g((unsigned)((a.N + 255) / 256));
    if (precision == PD_PREC_FP64)
        hipLaunchKernelGGL(k_cl_contact<double>, g, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_cl_contact<float>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rc_fused(const DevArgs &a, const ClArgs &c, const MlpArgs &m, int precision,
                           bool learned, bool list, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!(a.cl_on && a.cl_fx && a.cl_fy && c.rs && c.qr && c.qv && c.qa && c.qrb && c.alist && c.acnt &&
          c.Mt && c.I0 && c.bvec && c.phimax && c.rmax && c.rb_shape && c.rb_first && c.rb_count &&
          c.n_rb > 0))
        return hipErrorInvalidValue;
    if (learned && !(m.wfr && m.wf && m.sig_q && m.sig_r && m.lam)) return hipErrorInvalidValue;
    const dim3 g((unsigned)c.n_rb), b(64 * kRcWaves);
    const int li = list ? 1 : 0;
    if (precision == PD_PREC_FP64) {
        if (learned)
            hipLaunchKernelGGL((k_rc_fused<double, true, kRcWaves>), g, b, 0, s, a, c, m, li);
        else
            hipLaunchKernelGGL((k_rc_fused<double, false, kRcWaves>), g, b, 0, s, a, c, m, li);
    } else {
        if (learned)
            hipLaunchKernelGGL((k_rc_fused<float, true, kRcWaves>), g, b, 0, s, a, c, m, li);
        else
            hipLaunchKernelGGL((k_rc_fused<float, false, kRcWaves>), g, b, 0, s, a, c, m, li);
    }
    return hipGetLastError();
}

// At a list rebuild (positions advanced as the lists were built), the active
// nodes of closure particles: those with contact candidates, the candidates
// of any node, and those within the list radius of a wall of their
// aggregate.  Until the next rebuild no other node can come within R_c of
// anything: nodes move less than half the skin between rebuilds (the lists'
// own rule, a bound on the rigid + modal motion for reduced particles) and
// the top wall is held to half the skin as well.
__global__ void k_rc_mark(DevArgs a, uint8_t *act, double t_next) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int pi = a.part[i];
    const bool mine = a.cl_on[pi] != 0;
    const int n = a.clist_n[i];
    if (mine) {
        double px, py, ux, uy;
        advanced_pos(a, i, true, px, py, ux, uy);
        const int ag = a.pagg[pi];
        const double *b = a.box + 4 * ag;
        const double top = b[3] - a.vtop[ag] * t_next;
        const double rl = sqrt(a.Rl2);
        if (n > 0 || px - b[0] < rl || b[1] - px < rl || py - b[2] < rl || top - py < rl) act[i] = 1;
    }
    for (int k = 0; k < n; ++k) {
        const int j = (int)a.clist[(size_t)k * a.N + i];
        if (a.cl_on[a.part[j]]) act[j] = 1;
    }
}

hipError_t launch_rc_mark(const DevArgs &a, uint8_t *act, double t_next, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    if (!(a.cl_on && a.clist && a.clist_n && act)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rc_mark, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, a, act, t_next);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the pass of list-mode steps (closure off): the code of the walls and of
// the contact candidates needs more registers than the rest of the step
// kernel, so for large problems it runs in a launch of its own over the few
// nodes near a wall or with candidates, and the step kernel, which then
// reads the results, keeps more wavefronts in flight
// ---------------------------------------------------------------------------
// at a list rebuild (positions advanced as the lists were built): every node
// within the list radius of a wall of its aggregate (the top wall at the time
// of the step after *step_base, the rebuild's step), or beyond one, onto the
// wall list; every node with contact candidates onto the contact list (a
// node that gets its first candidates from a broken bond later joins it from
// the step kernel).  Until the next rebuild no other node can come within
// R_c of a wall: nodes move less than half the skin between rebuilds, and
// the top wall is held to half the skin as well.
__global__ void k_pass_mark(DevArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const double t_next = (double)(*a.step_base + 1) * a.dt;
    double px, py, ux, uy;
    advanced_pos(a, i, true, px, py, ux, uy);
    const int ag = a.pagg[a.part[i]];
    const double *b = a.box + 4 * ag;
    const double top = b[3] - a.vtop[ag] * t_next;
    const double rl = sqrt(a.Rl2);
    if (px - b[0] < rl || b[1] - px < rl || py - b[2] < rl || top - py < rl) {
        const unsigned long long k = atomicAdd(a.wall_n, 1ull);
        a.wall_list[k] = i;
    }
    if (a.clist_n[i] > 0) a.cont_list[atomicAdd(a.cont_n, 1ull)] = i;
}

// The pass before each list-mode step kernel: at the position and velocity
// the step kernel uses, each listed node's wall force (a quad per node, a
// lane per wall region, summed as the step kernel's four lanes sum them, so
// the result is the same whatever its lane count), then each listed node's contact
// forces over its candidates (LPN lanes per node, the step kernel's lanes and
// order: the same bits).  A launch past the first stale step of a replay does
// nothing.
template <typename R, int LPN>
__global__ __launch_bounds__(256) void k_pass(DevArgs a) {
    const long long sprev = *a.step_base + a.chunk_k;
    if ((unsigned long long)(sprev + 1) >= *a.invalid_step) return;
    const bool un = a.chunk_k > 0 && a.unx && !a.cl_on;
    const double t = (double)(sprev + 1) * a.dt;
    // even workgroups take the wall list, odd ones the contact list (the two
    // chains of dependent work side by side rather than one after the other)
    const long long stride = (long long)(gridDim.x / 2) * blockDim.x;
    const long long tid = (long long)(blockIdx.x / 2) * blockDim.x + threadIdx.x;
    const long long n = (blockIdx.x & 1) ? 0 : (long long)*a.wall_n;
    // walls: the four lanes of a quad per listed node, lane r the wall region
    // r, summed (l0 + l1) + (l2 + l3) as the four-lane step kernel sums them
    const int r = (int)(threadIdx.x & 3);
    for (long long k = tid >> 2; k < n; k += stride >> 2) {
        const int i = a.wall_list[k];
        double pxi, pyi, uxi, uyi;
        advanced_pos_un(a, i, un, pxi, pyi, uxi, uyi);
        const int pi = a.part[i];
        const int ag = a.pagg[pi];
        const MatConst mc = a.mat[a.pmat[pi]];
        const double Vi = a.vol[i], mi = mc.rho * Vi;
        const double vxi = a.vx[i], vyi = a.vy[i];
        int st = 0;
        double fx = 0.0, fy = 0.0;
        wall_forces(a, ag, r, pxi, pyi, vxi, vyi, mi, Vi, mc.Kn, t, fx, fy, st);
        fx = lanes_sum<4>(fx);
        fy = lanes_sum<4>(fy);
        st = lanes_or<4>(st);
        if (r == 0) {
            a.wfx[i] = fx;
            a.wfy[i] = fy;
            if (st) atomicOr(a.status, st);
        }
    }
    const long long nc = (blockIdx.x & 1) ? (long long)*a.cont_n : 0;
    const int sub = (int)(threadIdx.x & (LPN - 1));
    for (long long k = tid / LPN; k < nc; k += stride / LPN) {
        const int i = a.cont_list[k];
        const int pi = a.part[i];
        const MatConst mc = a.mat[a.pmat[pi]];
        const double xi = a.x[i], yi = a.y[i];
        double pxi, pyi, uxi, uyi;
        advanced_pos_un(a, i, un, pxi, pyi, uxi, uyi);
        const double vxi = a.vx[i], vyi = a.vy[i];
        const double Vi = a.vol[i], mi = mc.rho * Vi;
        R fsx = 0, fsy = 0, fnx = 0, fny = 0;
        contact_forces<R, true, true, LPN>(a, mc, i, sub, pi, a.pagg[pi], xi, yi, pxi, pyi, vxi,
                                           vyi, Vi, mi, fsx, fsy, fnx, fny, a.clist_n[i], un);
        fsx = lanes_sum<LPN>(fsx);
        fsy = lanes_sum<LPN>(fsy);
        fnx = lanes_sum<LPN>(fnx);
        fny = lanes_sum<LPN>(fny);
        if (sub == 0) {
            *reinterpret_cast<double2 *>(a.csum + 4 * (size_t)i) = make_double2(fsx, fsy);
            *reinterpret_cast<double2 *>(a.csum + 4 * (size_t)i + 2) = make_double2(fnx, fny);
        }
    }
}

hipError_t launch_pass_mark(const DevArgs &a, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    if (!(a.wall_list && a.wall_n && a.cont_list && a.cont_n)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pass_mark, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename R>
static void launch_pass_t(const DevArgs &a, int lpn, unsigned g, hipStream_t s) {
    if (lpn == 1)
        hipLaunchKernelGGL((k_pass<R, 1>), dim3(g), dim3(256), 0, s, a);
    else if (lpn == 2)
        hipLaunchKernelGGL((k_pass<R, 2>), dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_pass<R, 4>), dim3(g), dim3(256), 0, s, a);
}

hipError_t launch_pass(const DevArgs &a, int precision, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    if (!(a.wall_list && a.wall_n && a.wfx && a.wfy && a.cont_list && a.cont_n && a.csum))
        return hipErrorInvalidValue;
    if (!(a.lanes == 1 || a.lanes == 2 || a.lanes == 4)) return hipErrorInvalidValue;
    // a fixed grid (the lists' lengths change at rebuilds and appends,
    // replays keep the grid they were captured with), an even number of
    // workgroups (half for each list), two per compute unit
    const unsigned g = 2u * std::min<unsigned>((unsigned)((a.N + 511) / 512), 256u);
    if (precision == PD_PREC_FP64)
        launch_pass_t<double>(a, a.lanes, g, s);
    else
        launch_pass_t<float>(a, a.lanes, g, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction observables (Sec. 7.4): wall reactions, bond counts, damage
// ---------------------------------------------------------------------------
// each wall's share of the wall force on node i at the current state
// (positions x + u, velocities v, top wall at t = step dt): a wall segment
// counts for its wall, a corner correction half for each of its two walls
__global__ void k_wall_split(DevArgs a, double *split) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int pi = a.part[i];
    const int ag = a.pagg[pi];
    const MatConst mc = a.mat[a.pmat[pi]];
    const double px = a.x[i] + a.ux[i], py = a.y[i] + a.uy[i];
    const double t = (double)(*a.step) * a.dt;
    double w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int pa[4] = {0, 2, 1, 3}, pb[4] = {2, 1, 3, 0};
    int st = 0;
    for (int part = 0; part < 4; ++part) {
        double sgx = 0.0, sgy = 0.0, crx = 0.0, cry = 0.0;
        wall_parts(a, ag, part, px, py, a.vx[i], a.vy[i], a.mass[i], a.vol[i], mc.Kn, t, sgx, sgy,
                   crx, cry, st);
        w[2 * part] += sgx;
        w[2 * part + 1] += sgy;
        w[2 * pa[part]] += 0.5 * crx;
        w[2 * pa[part] + 1] += 0.5 * cry;
        w[2 * pb[part]] += 0.5 * crx;
        w[2 * pb[part] + 1] += 0.5 * cry;
    }
    for (int k = 0; k < 8; ++k) split[(size_t)k * a.N + i] = w[k];
}

// per aggregate (one workgroup each, over its particles in order): minus the
// sum of the walls' shares (the force on each wall), broken and reference
// directed bonds; out[10 a + k]
__global__ __launch_bounds__(256) void k_obs_reduce(DevArgs a, const double *split,
                                                    const int *agg_pstart, const int *agg_parts,
                                                    const int *poff, double *out) {
    __shared__ double sh[4 * 10];
    const int ag = blockIdx.x;
    double v[10];
    for (int k = 0; k < 10; ++k) v[k] = 0.0;
    for (int q = agg_pstart[ag]; q < agg_pstart[ag + 1]; ++q) {
        const int p = agg_parts[q];
        for (int i = poff[p] + threadIdx.x; i < poff[p + 1]; i += 256) {
            for (int k = 0; k < 8; ++k) v[k] -= split[(size_t)k * a.N + i];
            const uint32_t sl = (uint32_t)i / kSlice;
            const uint32_t base = a.slice_ptr[sl] + (uint32_t)i % kSlice;
            const int W = (int)((a.slice_ptr[sl + 1] - a.slice_ptr[sl]) / kSlice);
            for (int k = 0; k < W; ++k) {
                const uint32_t e = a.col[base + (uint32_t)k * kSlice];
                if ((int)(e & kIndexMask) == i) continue;  // padding
                v[9] += 1.0;
                if (e & kBroken) v[8] += 1.0;
            }
        }
    }
    for (int k = 0; k < 10; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 10; ++k) sh[w * 10 + k] = v[k];
    __syncthreads();
    if (threadIdx.x < 10) {
        const int k = threadIdx.x;
        out[10 * ag + k] = ((sh[k] + sh[10 + k]) + sh[20 + k]) + sh[30 + k];
    }
}

// broken / reference directed bonds of each particle (one workgroup each)
__global__ __launch_bounds__(256) void k_particle_damage(DevArgs a, const int *poff, double *out) {
    __shared__ unsigned sh[8];
    const int p = blockIdx.x;
    unsigned nb = 0, nr = 0;
    for (int i = poff[p] + threadIdx.x; i < poff[p + 1]; i += 256) {
        const uint32_t sl = (uint32_t)i / kSlice;
        const uint32_t base = a.slice_ptr[sl] + (uint32_t)i % kSlice;
        const int W = (int)((a.slice_ptr[sl + 1] - a.slice_ptr[sl]) / kSlice);
        for (int k = 0; k < W; ++k) {
            const uint32_t e = a.col[base + (uint32_t)k * kSlice];
            if ((int)(e & kIndexMask) == i) continue;
            ++nr;
            if (e & kBroken) ++nb;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        nb += __shfl_xor(nb, o, 64);
        nr += __shfl_xor(nr, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[2 * w] = nb;
        sh[2 * w + 1] = nr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned b = sh[0] + sh[2] + sh[4] + sh[6], r = sh[1] + sh[3] + sh[5] + sh[7];
        out[p] = r ? (double)b / (double)r : 0.0;
    }
}

// ---------------------------------------------------------------------------
// fragments: connected components of the intact-bond graph (the child
// particles of Sec. 7.3).  Labels only ever decrease and always name a node
// of the same component, so the fixed point is the smallest node index of
// each component whatever the order of the updates.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ld_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_cc_init(int *L, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) L[i] = i;
}

// every node takes the smallest label among itself and its intact partners,
// hooks its current label onto it, and pushes it to partners that hold a
// larger one (so a bond joins its nodes if either directed copy is intact)
__global__ __launch_bounds__(256) void k_cc_hook(DevArgs a, int *L, int *changed) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.N) return;
    const int li = ld_relaxed(L + i);
    int m = li, top = li;
    const uint32_t sl = (uint32_t)i / kSlice;
    const uint32_t base = a.slice_ptr[sl] + (uint32_t)i % kSlice;
    const int W = (int)((a.slice_ptr[sl + 1] - a.slice_ptr[sl]) / kSlice);
    for (int k = 0; k < W; ++k) {
        const uint32_t e = a.col[base + (uint32_t)k * kSlice];
        const int j = (int)(e & kIndexMask);
        if (j == i || (e & kBroken)) continue;
        const int lj = ld_relaxed(L + j);
        m = min(m, lj);
        top = max(top, lj);
    }
    if (m < li) {
        atomicMin(L + i, m);
        atomicMin(L + li, m);
    }
    const bool push = top > m;
    if (push) {
        for (int k = 0; k < W; ++k) {
            const uint32_t e = a.col[base + (uint32_t)k * kSlice];
            const int j = (int)(e & kIndexMask);
            if (j == i || (e & kBroken)) continue;
            const int lj = ld_relaxed(L + j);
            if (lj > m) {
                atomicMin(L + j, m);
                atomicMin(L + lj, m);
            }
        }
    }
    if (m < li || push) atomicOr(changed, 1);
}

// pointer jumping: follow labels down to a node that names itself
__global__ __launch_bounds__(256) void k_cc_jump(int *L, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int v = ld_relaxed(L + i);
    for (;;) {  // strictly decreasing, so at most i rounds
        const int w = ld_relaxed(L + v);
        if (w >= v) break;
        v = w;
    }
    atomicMin(L + i, v);
}

// size[label] += 1 for every node
__global__ __launch_bounds__(256) void k_cc_size(const int *L, int *size, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) atomicAdd(size + L[i], 1);
}

// per particle, the components with at least min_nodes nodes; stats[0] counts all
__global__ __launch_bounds__(256) void k_cc_count(DevArgs a, const int *L, const int *size,
                                                  int min_nodes, int *count, int *stats) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.N || L[i] != i) return;
    atomicAdd(stats, 1);
    if (size[i] >= min_nodes) atomicAdd(count + a.part[i], 1);
}

hipError_t launch_cc_init(int *L, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cc_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L, n);
    return hipGetLastError();
}

hipError_t launch_cc_round(const DevArgs &a, int *L, int *changed, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    const dim3 g((unsigned)((a.N + 255) / 256));
    hipLaunchKernelGGL(k_cc_hook, g, dim3(256), 0, s, a, L, changed);
    hipLaunchKernelGGL(k_cc_jump, g, dim3(256), 0, s, L, a.N);
    return hipGetLastError();
}

hipError_t launch_cc_count(const DevArgs &a, const int *L, int *size, int min_nodes, int *count,
                           int *stats, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    const dim3 g((unsigned)((a.N + 255) / 256));
    hipLaunchKernelGGL(k_cc_size, g, dim3(256), 0, s, L, size, a.N);
    hipLaunchKernelGGL(k_cc_count, g, dim3(256), 0, s, a, L, size, min_nodes, count, stats);
    return hipGetLastError();
}

hipError_t launch_observables(const DevArgs &a, double *split, const int *agg_pstart,
                              const int *agg_parts, const int *poff, double *out, hipStream_t s) {
    DevArgs b = a;
    b.counting = 0;  // an observation, not a step: no event counts
    hipLaunchKernelGGL(k_wall_split, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, s, b, split);
    hipLaunchKernelGGL(k_obs_reduce, dim3(a.A), dim3(256), 0, s, b, split, agg_pstart, agg_parts, poff,
                       out);
    return hipGetLastError();
}

hipError_t launch_particle_damage(const DevArgs &a, const int *poff, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_particle_damage, dim3(a.P), dim3(256), 0, s, a, poff, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------
__global__ void k_sum_terms(DevArgs a, uint32_t mask, double *fx, double *fy) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    double sx = 0.0, sy = 0.0;
    for (int t = 0; t < 5; ++t)
        if (mask & (1u << t)) {
            sx += a.terms[(2 * t) * a.N + i];
            sy += a.terms[(2 * t + 1) * a.N + i];
        }
    fx[i] = sx;
    fy[i] = sy;
}

__global__ void k_damage(DevArgs a, double *phi, unsigned long long *nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0, nref = 0;
    if (i < a.N) {
        const uint32_t base = a.slice_ptr[i / kSlice] + (uint32_t)(i % kSlice);
        nref = a.rowlen[i];
        for (int k = 0; k < nref; ++k) n += (a.col[base + (uint32_t)k * kSlice] & kBroken) ? 1 : 0;
        if (phi) phi[i] = nref > 0 ? (double)n / (double)nref : 0.0;
    }
    // wavefront reduction, one integer atomic per wavefront
    unsigned long long v = (unsigned long long)n;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(nb, v);
}

// contact set (pairs i < j) at the current sorted positions
template <bool FILL>
__global__ void k_contacts(DevArgs a, int *cnt, const long long *off, int *pi_out, int *pj_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    double pxi, pyi, ux, uy;
    advanced_pos(a, i, false, pxi, pyi, ux, uy);
    const int ag = a.pagg[a.part[i]];
    int cx, cy;
    cell_of(a, ag, pxi, pyi, cx, cy);
    const int ncx = a.agg_ncx[ag], ncy = a.agg_ncy[ag];
    long long w = FILL ? off[i] : 0;
    int n = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int yy = cy + dy, xx = cx + dx;
            if (yy < 0 || yy >= ncy || xx < 0 || xx >= ncx) continue;
            const uint32_t c = a.agg_cell0[ag] + (uint32_t)yy * (uint32_t)ncx + (uint32_t)xx;
            const uint32_t s = a.cell_start[c];
            if (s >= (uint32_t)a.N || a.skey[s] != c) continue;
            for (uint32_t k = s; k < (uint32_t)a.N && a.skey[k] == c; ++k) {
                const int j = a.perm[k];
                if (j <= i) continue;
                const double ddx = a.spx[k] - pxi, ddy = a.spy[k] - pyi;
                if (ddx * ddx + ddy * ddy < a.Rc2) {
                    if (FILL) {
                        pi_out[w] = i;
                        pj_out[w] = j;
                        ++w;
                    }
                    ++n;
                }
            }
        }
    if (!FILL) cnt[i] = n;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_bonds_count(const BondArgs &b, int *rowlen, uint8_t *row_full, hipStream_t s) {
    if (b.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bonds_count_w, dim3(grid_for(b.N, 128)), dim3(128), 0, s, b, rowlen,
                       row_full);
    return hipGetLastError();
}

hipError_t launch_node_broken(const DevArgs &a, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_broken, dim3(grid_for(a.N, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bonds_fill(const BondArgs &b, uint32_t *col, const uint32_t *slice_ptr,
                             hipStream_t s) {
    if (b.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bonds_fill_w, dim3(grid_for(b.N, 128)), dim3(128), 0, s, b, col,
                       slice_ptr);
    return hipGetLastError();
}

hipError_t launch_windows(const DevArgs &a, int *win_lo, int *win_hi, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_windows, dim3(grid_for(a.N, 256)), dim3(256), 0, s, a.col, a.slice_ptr,
                       a.rowlen, a.N, a.block_nodes, win_lo, win_hi);
    return hipGetLastError();
}

hipError_t launch_keys(const DevArgs &a, int adv, uint32_t *hist, int G, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    const unsigned g = grid_for(a.N, 256);
    if (hist && (sort_items(a.N) != 1 || (int)g != G)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_keys, dim3(g), dim3(256), 0, s, a, adv, hist, G);
    return hipGetLastError();
}

hipError_t launch_sort_pass(const uint32_t *kin, const int *vin, uint32_t *kout, int *vout, int N,
                            int shift, uint32_t *hist, uint32_t *dtotal, hipStream_t s,
                            hipEvent_t *ev, bool hist_done) {
    const int items = sort_items(N), G = sort_tiles(N);
    if (ev) hipEventRecord(ev[0], s);
    if (!hist_done)
        hipLaunchKernelGGL(k_hist, dim3(G), dim3(kSortBlock), 0, s, kin, N, shift, hist, G, items);
    if (ev) hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(k_digit_scan, dim3(kRadix), dim3(kSortBlock), 0, s, hist, G, dtotal);
    if (ev) hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(k_scatter, dim3(G), dim3(kSortBlock), 0, s, kin, vin, kout, vout, N, shift,
                       hist, G, dtotal, items);
    if (ev) hipEventRecord(ev[3], s);
    return hipGetLastError();
}

hipError_t launch_cells(const DevArgs &a, int adv, int advance_step, hipStream_t s) {
    const int n = a.N > 0 ? a.N : 1;
    hipLaunchKernelGGL(k_cells, dim3(grid_for(n, 256)), dim3(256), 0, s, a, adv, advance_step);
    return hipGetLastError();
}

int force_lds_cap(int max_win) { return max_win > kMaxLdsNodes ? 0 : max_win; }

template <typename R>
static void launch_force_t(const DevArgs &a, int mode, bool list, dim3 g, dim3 b, size_t shm,
                           hipStream_t s, int lds_cap, int sel, int lpn, bool wp) {
    if (mode == M_STEP) {
        if (list) {
            if (sel == 1)
                hipLaunchKernelGGL((k_force<R, M_STEP, true, 1>), g, b, 0, s, a, lds_cap);
            else if (wp && lpn == 1)
                hipLaunchKernelGGL((k_force_wp<R, 1>), g, b, shm, s, a, lds_cap);
            else if (wp && lpn == 2)
                hipLaunchKernelGGL((k_force_wp<R, 2>), g, b, shm, s, a, lds_cap);
            else if (wp)
                hipLaunchKernelGGL((k_force_wp<R, 4>), g, b, shm, s, a, lds_cap);
            else if (lpn == 1)
                hipLaunchKernelGGL((k_force<R, M_STEP, true, 0, 1>), g, b, shm, s, a, lds_cap);
            else if (lpn == 2)
                hipLaunchKernelGGL((k_force<R, M_STEP, true, 0, 2>), g, b, shm, s, a, lds_cap);
            else
                hipLaunchKernelGGL((k_force<R, M_STEP, true, 0>), g, b, shm, s, a, lds_cap);
        } else {
            hipLaunchKernelGGL((k_force<R, M_STEP, false, 0>), g, b, shm, s, a, lds_cap);
        }
    } else if (mode == M_FORCES) {
        hipLaunchKernelGGL((k_force<R, M_FORCES, false>), g, b, shm, s, a, lds_cap);
    } else {
        hipLaunchKernelGGL((k_force<R, M_PROLOGUE, false>), g, b, shm, s, a, lds_cap);
    }
}

hipError_t launch_force(const DevArgs &a, int precision, int mode, int lds_cap, hipStream_t s,
                        bool list, int sel, bool wall_pass) {
    if (a.N == 0) return hipSuccess;
    if (sel && !(mode == M_STEP && list && a.cl_on && a.pd_blocks && a.n_pd_blocks))
        return hipErrorInvalidValue;
    // the pass serves list-mode steps of the plain path only
    if (wall_pass && !(mode == M_STEP && list && !sel && !a.cl_on && a.wfx && a.wfy))
        return hipErrorInvalidValue;
    // nodes per workgroup, LPN lanes each (the tuning's lanes for list-mode
    // steps, four otherwise); the plain-force-only launch uses 64-node
    // workgroups (its list's unit), walks the list with a stride of at most
    // 1024 workgroups (four per compute unit) and stages nothing
    const int B = sel ? kSelBlockNodes : a.block_nodes;
    const int lpn = (mode == M_STEP && list && !sel) ? a.lanes : 4;
    if (!(lpn == 1 || lpn == 2 || lpn == 4) || lpn * B > 1024) return hipErrorInvalidValue;
    // the bond loop takes a wavefront's 64 / LPN nodes to be whole SELL-16 slices
    static_assert(kSelBlockNodes % kSlice == 0, "plain-force workgroups hold whole slices");
    if (B % kSlice != 0 || (64 / lpn) % kSlice != 0) return hipErrorInvalidValue;
    const size_t shm = (a.use_lds && !sel) ? (size_t)lds_cap * kWin * sizeof(double) : 0;
    const unsigned nb = (unsigned)grid_for(a.N, B);
    const dim3 g(sel ? std::min(nb, 1024u) : nb), b(lpn * B);
    if (precision == PD_PREC_FP64)
        launch_force_t<double>(a, mode, list, g, b, shm, s, lds_cap, sel, lpn, wall_pass);
    else
        launch_force_t<float>(a, mode, list, g, b, shm, s, lds_cap, sel, lpn, wall_pass);
    return hipGetLastError();
}

hipError_t launch_build_list(const DevArgs &a, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    if (a.maxc < 1 || a.maxc > kBlMaxc) return hipErrorInvalidValue;
    constexpr int kNodes = 64 / kBlLanes;
    const size_t shm = (size_t)kNodes * (size_t)a.maxc * sizeof(uint32_t);
    hipLaunchKernelGGL(k_build_list, dim3((unsigned)((a.N + kNodes - 1) / kNodes)), dim3(64), shm,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long *p, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_invalidate(const DevArgs &a, unsigned long long v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, a.invalid_step, v);
    return hipGetLastError();
}

hipError_t launch_round_start(const DevArgs &a, long long step, bool rebuild, hipStream_t s) {
    hipLaunchKernelGGL(k_round_start, dim3(1), dim3(1), 0, s, a, step, rebuild ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_arm_replay(const DevArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_arm_replay, dim3(1), dim3(1), 0, s, a.invalid_step, a.overflow);
    return hipGetLastError();
}

hipError_t launch_sum_terms(const DevArgs &a, uint32_t mask, double *fx, double *fy,
                            hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_terms, dim3(grid_for(a.N, 256)), dim3(256), 0, s, a, mask, fx, fy);
    return hipGetLastError();
}

hipError_t launch_damage(const DevArgs &a, double *phi, unsigned long long *nb, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_damage, dim3(grid_for(a.N, 256)), dim3(256), 0, s, a, phi, nb);
    return hipGetLastError();
}

hipError_t launch_contacts_count(const DevArgs &a, int *cnt, hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL((k_contacts<false>), dim3(grid_for(a.N, 256)), dim3(256), 0, s, a, cnt,
                       (const long long *)nullptr, (int *)nullptr, (int *)nullptr);
    return hipGetLastError();
}

hipError_t launch_contacts_fill(const DevArgs &a, const long long *off, int *pi, int *pj,
                                hipStream_t s) {
    if (a.N == 0) return hipSuccess;
    hipLaunchKernelGGL((k_contacts<true>), dim3(grid_for(a.N, 256)), dim3(256), 0, s, a,
                       (int *)nullptr, off, pi, pj);
    return hipGetLastError();
}

}  // namespace pd
