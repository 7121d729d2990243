// pd_closure.hip -- kernels of the learned modal closure.
//
// Nodal form (every node of a closure particle integrated each step):
//   k_cl_moments  one workgroup per closure particle: mass centroid, best-fit
//                 rotation (weighted 2-D Procrustes about the centroid),
//                 polar moment, angular velocity, total external force,
//                 torque and contact load
//   k_cl_modal,   particle blocks x 32-node slices with the slice's modes in
//   k_cl_modal_sum  LDS: q = Phi^T M u_body and the modal external force
//                 Phi^T f_body, then the slices summed in order
//   k_cl_apply    nodal accelerations of the rigid + modal motion,
//                 velocity-Verlet velocity update, the per-step gate
// Reduced form (centroid, angle and modal amplitudes integrated directly):
//   k_rc_init, k_rc_sync, k_rc_collect here; the step itself is one kernel,
//   k_rc_fused, beside the force kernel (it evaluates contact)
// Both:
//   k_mlp_fwd     the 32 -> 256 -> 256 -> 32 SiLU MLP on 16-row blocks, eight
//                 wavefronts splitting the columns, bfloat16 operands and
//                 float32 accumulation on the matrix cores (v_mfma 16x16x32
//                 bf16), weights read in fragment order, hidden activations
//                 in LDS
//   k_mlp_pack    a shape's weights into that fragment order (after every
//                 change of the weights)
//   k_cl_check_part, k_cl_check_sum: the periodic check against the plain force
//   k_gemm        strided bf16 GEMM on the matrix cores (training backward)
//   k_mlp_loss, k_colsum, k_adam, k_mlp_init, k_batch_idx, k_norm_stats:
//                 the rest of a training iteration
//
// The paper has no reduced-order model; the closure replaces the bond force
// of eq. (peri) for particles far from the break threshold of Sec. 3.1 and
// under light contact, and the plain bond force stays the fallback and the
// periodic check.
#include <math.h>

#include "pd_closure_dev.h"
#include "pd_mlp_dev.h"

namespace pd {

__device__ __forceinline__ double block_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// ---------------------------------------------------------------------------
// projection on the rigid + modal coordinates, in two kernels
//
// mode 0 (step):  positions x + u_o (the advanced displacement the force
//                 kernel wrote), velocities v (previous step), forces cl_fx/fy
// mode 1 (check): positions x + u (current state), forces terms[PD] * V, for
//                 active particles; gext then holds the modal PD force
// mode 2 (snapshot): as 1, for every closure particle
// ---------------------------------------------------------------------------
__device__ __forceinline__ void node_force(const DevArgs &a, int mode, int i, double &fx,
                                           double &fy) {
    if (mode == 0) {
        fx = a.cl_fx[i];
        fy = a.cl_fy[i];
    } else {
        fx = a.terms[i] * a.vol[i];
        fy = a.terms[a.N + i] * a.vol[i];
    }
}

// k_cl_moments: one workgroup per closure particle, one pass over its nodes:
// moments about the particle's first node give the centroid, the Procrustes
// sums (the template coordinates are centred), the polar moment, the angular
// momentum, the total force, the torque and the contact load
__global__ __launch_bounds__(256) void k_cl_moments(DevArgs a, ClArgs c, int list, int mode) {
    __shared__ double red[4 * 16];
    if (replay_stale(a, list && mode == 0)) return;
    const int ci = blockIdx.x;
    const int p = c.cpart[ci];
    if (mode < 2 && !a.cl_on[p]) {
        if (threadIdx.x == 0) c.red[(size_t)ci * 16 + R_ACTIVE] = 0.0;
        return;
    }
    const int s = c.cshape[ci];
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    const int t0 = c.toff[s];
    const double *ux = mode == 0 ? a.ux_o : a.ux;
    const double *uy = mode == 0 ? a.uy_o : a.uy;
    const double rx = a.x[n0] + ux[n0], ry = a.y[n0] + uy[n0];
    double v[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) v[k] = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        const int i = n0 + k;
        const double m = a.mass[i];
        const double yx = (a.x[i] + ux[i]) - rx, yy = (a.y[i] + uy[i]) - ry;
        const double vx = a.vx[i], vy = a.vy[i];
        double fx, fy;
        node_force(a, mode, i, fx, fy);
        const double Xx = c.tX[t0 + k], Xy = c.tY[t0 + k];
        v[0] += m;
        v[1] += m * yx;
        v[2] += m * yy;
        v[3] += m * vx;
        v[4] += m * vy;
        v[5] += fx;
        v[6] += fy;
        v[7] += m * (Xx * yy - Xy * yx);
        v[8] += m * (Xx * yx + Xy * yy);
        v[9] += m * (yx * yx + yy * yy);
        v[10] += m * (yx * vy - yy * vx);
        v[11] += yx * fy - yy * fx;
        v[12] += sqrt(fx * fx + fy * fy);
        v[13] += m * Xx;
        v[14] += m * Xy;
    }
    block_sum<15>(v, red);
    if (threadIdx.x != 0) return;
    const double M = v[0];
    const double cx = v[1] / M, cy = v[2] / M;  // centroid, relative to the first node
    const double vcx = v[3] / M, vcy = v[4] / M;
    const double Ftx = v[5], Fty = v[6];
    const double cross = v[7] - (v[13] * cy - v[14] * cx);
    const double dot = v[8] - (v[13] * cx + v[14] * cy);
    const double I = v[9] - M * (cx * cx + cy * cy);
    const double Lz = v[10] - M * (cx * vcy - cy * vcx);
    const double tau = v[11] - (cx * Fty - cy * Ftx);
    // the best-fit rotation: (cos, sin) = (dot, cross) / |(dot, cross)|
    const double nr = sqrt(dot * dot + cross * cross);
    double *R = c.red + (size_t)ci * 16;
    R[R_M] = M;
    R[R_CX] = rx + cx;
    R[R_CY] = ry + cy;
    R[R_VCX] = vcx;
    R[R_VCY] = vcy;
    R[R_PHI] = 0.0;
    R[R_COS] = dot / nr;
    R[R_SIN] = cross / nr;
    R[R_I] = I;
    R[R_OM] = Lz / I;
    R[R_FX] = Ftx;
    R[R_FY] = Fty;
    R[R_TAU] = tau;
    R[R_CONTACT] = v[12];
    R[R_ACTIVE] = 1.0;
}

// k_cl_modal: one workgroup per (block of up to 16 closure particles of one
// shape, 32-node slice of the shape).  The slice's modes and every
// particle's m u_body and f_body on it are staged in LDS; thread (particle p,
// mode k) adds the slice's terms of q_pk = (Phi^T M u_body)_k and
// gext_pk = (Phi^T f_body)_k, and leaves them in part[]; k_cl_modal_sum adds
// the slices in order.  Each staged mode entry serves 16 particles.
constexpr int kModalSlice = 32;

__global__ __launch_bounds__(512) void k_cl_modal(DevArgs a, ClArgs c, int list, int mode) {
    __shared__ float2 Ph[kModalSlice][kClModes];
    __shared__ double4 U[16][kModalSlice];
    __shared__ double Rs[16][4];
    __shared__ int pn0[16], pok[16];
    if (replay_stale(a, list && mode == 0)) return;
    const int rb = blockIdx.x, sl = blockIdx.y;
    const int s = c.rb_shape[rb], first = c.rb_first[rb], cnt = c.rb_count[rb];
    const int t0 = c.toff[s];
    const int n = c.poff[c.cpart[first] + 1] - c.poff[c.cpart[first]];
    const int j0 = sl * kModalSlice;
    if (j0 >= n) return;  // a slice past this shape's nodes (uniform)
    const int tid = threadIdx.x;
    if (tid < 16) {
        int ok = 0, n0 = 0;
        if (tid < cnt) {
            const int p = c.cpart[first + tid];
            ok = mode == 2 || a.cl_on[p];
            n0 = c.poff[p];
            const double *R = c.red + (size_t)(first + tid) * 16;
            Rs[tid][0] = R[R_CX];
            Rs[tid][1] = R[R_CY];
            Rs[tid][2] = R[R_COS];
            Rs[tid][3] = R[R_SIN];
        }
        pok[tid] = ok;
        pn0[tid] = n0;
    }
    __syncthreads();
    const double *ux = mode == 0 ? a.ux_o : a.ux;
    const double *uy = mode == 0 ? a.uy_o : a.uy;
    const float2 *phi2 = reinterpret_cast<const float2 *>(c.phi);
    for (int e = tid; e < kModalSlice * kClModes; e += 512) {
        const int jj = e / kClModes, kk = e % kClModes;
        Ph[jj][kk] = j0 + jj < n ? phi2[(size_t)(t0 + j0 + jj) * kClModes + kk]
                                 : make_float2(0.f, 0.f);
    }
    {
        const int q = tid / kModalSlice, jj = tid % kModalSlice;  // 16 x 32 = 512
        double4 w = make_double4(0.0, 0.0, 0.0, 0.0);
        if (pok[q] && j0 + jj < n) {
            const int i = pn0[q] + j0 + jj;
            const double m = a.mass[i];
            const double Yx = (a.x[i] + ux[i]) - Rs[q][0], Yy = (a.y[i] + uy[i]) - Rs[q][1];
            const double cp = Rs[q][2], sp = Rs[q][3];
            double fx, fy;
            node_force(a, mode, i, fx, fy);
            w.x = m * ((cp * Yx + sp * Yy) - c.tX[t0 + j0 + jj]);
            w.y = m * ((-sp * Yx + cp * Yy) - c.tY[t0 + j0 + jj]);
            w.z = cp * fx + sp * fy;
            w.w = -sp * fx + cp * fy;
        }
        U[q][jj] = w;
    }
    __syncthreads();
    const int pp = tid >> 5, k = tid & 31;
    if (pp >= cnt || !pok[pp]) return;
    double sq = 0.0, sf = 0.0;
    const int jn = min(kModalSlice, n - j0);
    for (int jj = 0; jj < jn; ++jj) {
        const float2 f = Ph[jj][k];
        const double4 w = U[pp][jj];
        sq += (double)f.x * w.x + (double)f.y * w.y;
        sf += (double)f.x * w.z + (double)f.y * w.w;
    }
    double *out = c.part + (((size_t)(first + pp) * c.n_slices + sl) * kClModes + k) * 2;
    out[0] = sq;
    out[1] = sf;
}

// the slices' parts in order: q, gext and the stretch bound of each particle
__global__ __launch_bounds__(256) void k_cl_modal_sum(DevArgs a, ClArgs c, int list, int mode) {
    if (replay_stale(a, list && mode == 0)) return;
    const int ci = blockIdx.x * 8 + (threadIdx.x >> 5), k = threadIdx.x & 31;
    if (ci >= c.Pc) return;
    const int p = c.cpart[ci];
    if (mode < 2 && !a.cl_on[p]) return;
    const int s = c.cshape[ci];
    const int n = c.poff[p + 1] - c.poff[p];
    const int ns = (n + kModalSlice - 1) / kModalSlice;
    const double *in = c.part + ((size_t)ci * c.n_slices * kClModes + k) * 2;
    double sq = 0.0, sf = 0.0;
    for (int sl = 0; sl < ns; ++sl) {
        sq += in[(size_t)sl * kClModes * 2];
        sf += in[(size_t)sl * kClModes * 2 + 1];
    }
    c.q[ci * kClModes + k] = sq;
    c.gext[ci * kClModes + k] = sf;
    // first-order bound of the largest bond stretch, sum_k |q_k| sigma_k
    double b = fabs(sq) * c.sig[s * kClModes + k];
    for (int o = 16; o > 0; o >>= 1) b += __shfl_xor(b, o, 32);
    if (k == 0) c.red[(size_t)ci * 16 + R_STRAIN] = b;
}

// ---------------------------------------------------------------------------
// nodal accelerations of the rigid + modal motion, velocity update, gate
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_cl_apply(DevArgs a, ClArgs c, int list) {
    __shared__ float2 PhT[kClModes][kModalSlice];  // mode-major: lanes of one mode are conflict-free
    __shared__ double Qd[16][kClModes];
    __shared__ double Rs[16][16];
    __shared__ int pn0[16], pok[16];
    if (replay_stale(a, list)) return;
    const int rb = blockIdx.x, sl = blockIdx.y;
    const int s = c.rb_shape[rb], first = c.rb_first[rb], cnt = c.rb_count[rb];
    const int t0 = c.toff[s];
    const int n = c.poff[c.cpart[first] + 1] - c.poff[c.cpart[first]];
    const int j0 = sl * kModalSlice;
    if (j0 >= n) return;  // uniform
    const int tid = threadIdx.x;
    // which particles step under the closure was fixed by k_cl_moments
    // (the gate below may clear cl_on while other slices still run)
    if (tid < 16) {
        int ok = 0;
        if (tid < cnt) ok = c.red[(size_t)(first + tid) * 16 + R_ACTIVE] != 0.0;
        pok[tid] = ok;
        pn0[tid] = tid < cnt ? c.poff[c.cpart[first + tid]] : 0;
    }
    {
        const int q = tid >> 5, k = tid & 31;  // 16 x 32
        if (q < cnt) {
            const int ci = first + q;
            const double qq = c.q[ci * kClModes + k];
            const double g = c.learned ? c.ghat[ci * kClModes + k] : -c.lam[s * kClModes + k] * qq;
            Qd[q][k] = g + c.gext[ci * kClModes + k];
            if (k < 16) Rs[q][k] = c.red[(size_t)ci * 16 + k];
        }
        const int jj = tid >> 4, kk2 = (tid & 15) * 2;  // 32 nodes x 16 mode pairs
        const float4 f = j0 + jj < n
                             ? reinterpret_cast<const float4 *>(c.phi + (size_t)(t0 + j0 + jj) * 2 * kClModes)[kk2 / 2]
                             : make_float4(0.f, 0.f, 0.f, 0.f);
        PhT[kk2][jj] = make_float2(f.x, f.y);
        PhT[kk2 + 1][jj] = make_float2(f.z, f.w);
    }
    __syncthreads();
    const int q = tid >> 5, jj = tid & 31;
    int st = 0;
    int stale = 0;
    if (q < cnt && pok[q] && j0 + jj < n) {
        double bx = 0.0, by = 0.0;
#pragma unroll 8
        for (int k = 0; k < kClModes; ++k) {
            const float2 f = PhT[k][jj];
            bx += (double)f.x * Qd[q][k];
            by += (double)f.y * Qd[q][k];
        }
        const double *R = Rs[q];
        const double M = R[R_M], cx = R[R_CX], cy = R[R_CY];
        const double cp = R[R_COS], sp = R[R_SIN];
        const double alpha = R[R_TAU] / R[R_I], om2 = R[R_OM] * R[R_OM];
        const double atx = R[R_FX] / M + a.gx, aty = R[R_FY] / M + a.gy;
        const int i = pn0[q] + j0 + jj;
        const double ux = a.ux_o[i], uy = a.uy_o[i];
        const double Yx = (a.x[i] + ux) - cx, Yy = (a.y[i] + uy) - cy;
        const double axn = ((atx - alpha * Yy) - om2 * Yx) + (cp * bx - sp * by);
        const double ayn = ((aty + alpha * Yx) - om2 * Yy) + (sp * bx + cp * by);
        const double vxn = a.vx[i] + a.hdt * (a.ax[i] + axn);
        const double vyn = a.vy[i] + a.hdt * (a.ay[i] + ayn);
        a.ax_o[i] = axn;
        a.ay_o[i] = ayn;
        a.vx_o[i] = vxn;
        a.vy_o[i] = vyn;
        if (!(isfinite(vxn) && isfinite(vyn))) st |= kStNonfinite;
        if (list) {
            const double unx = (ux + a.dt * vxn) + a.hdt2 * axn;
            const double uny = (uy + a.dt * vyn) + a.hdt2 * ayn;
            const double ex = unx - (double)a.ubx[i], ey = uny - (double)a.uby[i];
            if (!(ex * ex + ey * ey <= a.move2)) stale = 1;
        }
    }
    if (st) atomicOr(a.status, st);
    if (__syncthreads_or(stale) && tid == 0) {
        const long long sprev = *a.step_base + a.chunk_k;
        atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));
    }
    // gate for the next step (once per particle, by the first slice): a
    // particle whose bound on the bond stretch passes gate_frac * s0, or
    // whose contact load passes tau_c, goes back to the plain bond force
    if (sl == 0 && jj == 0 && q < cnt && pok[q]) {
        const double *R = Rs[q];
        if (R[R_STRAIN] > c.gate_frac * c.s0[s] || R[R_CONTACT] > c.tau_c[s]) {
            const int p = c.cpart[first + q];
            a.cl_on[p] = 0;
            list_particle_blocks(a, c, p);
            atomicAdd(c.fallbacks, 1ull);
        }
    }
}

// ---------------------------------------------------------------------------
// reduced mode: a closure particle's state is its centroid c, rotation angle
// phi about the template orientation and modal amplitudes q, with their rates
// and accelerations, integrated by velocity Verlet.  A node's position is
// c + R(phi) (X + Phi q), its velocity and acceleration follow by
// differentiation (without the Coriolis term of the modal rate, as in the
// nodal form).  A step handles only the particle's active nodes (listed at the
// last list rebuild: the only ones that can meet other nodes or walls before
// the next); every node is reconstructed before anything reads the nodal
// state.
// ---------------------------------------------------------------------------
// k_rc_init: the reduced state of every active closure particle from the
// current nodal state: centroid, velocity and acceleration of the mass
// centroid; the best-fit angle; angular velocity and acceleration from the
// angular momentum and its rate about the centroid; q, its rate and its
// acceleration as projections of the body-frame deformation, velocity and
// acceleration left after the rigid motion
__global__ __launch_bounds__(256) void k_rc_init(DevArgs a, ClArgs c) {
    __shared__ double red[4 * 14];
    __shared__ double part[8][kClModes][3];
    const int ci = blockIdx.x;
    const int p = c.cpart[ci];
    if (!a.cl_on[p]) return;
    const int s = c.cshape[ci];
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    const int t0 = c.toff[s];
    const double rx = a.x[n0] + a.ux[n0], ry = a.y[n0] + a.uy[n0];
    double v[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) v[k] = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const int i = n0 + j;
        const double m = a.mass[i];
        const double yx = (a.x[i] + a.ux[i]) - rx, yy = (a.y[i] + a.uy[i]) - ry;
        const double Xx = c.tX[t0 + j], Xy = c.tY[t0 + j];
        v[0] += m;
        v[1] += m * yx;
        v[2] += m * yy;
        v[3] += m * a.vx[i];
        v[4] += m * a.vy[i];
        v[5] += m * a.ax[i];
        v[6] += m * a.ay[i];
        v[7] += m * (Xx * yy - Xy * yx);
        v[8] += m * (Xx * yx + Xy * yy);
        v[9] += m * (yx * yx + yy * yy);
        v[10] += m * (yx * a.vy[i] - yy * a.vx[i]);
        v[11] += m * (yx * a.ay[i] - yy * a.ax[i]);
        v[12] += m * Xx;
        v[13] += m * Xy;
    }
    block_sum<14>(v, red);
    const double M = v[0];
    const double cx = v[1] / M, cy = v[2] / M;  // about the first node
    const double vcx = v[3] / M, vcy = v[4] / M, acx = v[5] / M, acy = v[6] / M;
    const double cross = v[7] - (v[12] * cy - v[13] * cx);
    const double dot = v[8] - (v[12] * cx + v[13] * cy);
    const double I = v[9] - M * (cx * cx + cy * cy);
    const double om = (v[10] - M * (cx * vcy - cy * vcx)) / I;
    const double al = (v[11] - (cx * v[6] - cy * v[5])) / I;
    const double phi = atan2(cross, dot);
    const double cp = cos(phi), sp = sin(phi), om2 = om * om;
    const double Cx = rx + cx, Cy = ry + cy;
    if (threadIdx.x == 0) {
        double *R = c.rs + (size_t)ci * 16;
        R[RS_CX] = Cx;
        R[RS_CY] = Cy;
        R[RS_VX] = vcx;
        R[RS_VY] = vcy;
        R[RS_AX] = acx;
        R[RS_AY] = acy;
        R[RS_PHI] = phi;
        R[RS_OM] = om;
        R[RS_AL] = al;
    }
    // projections, thread (mode k, part of the nodes)
    const int k = threadIdx.x & 31, pt = threadIdx.x >> 5;
    double sq = 0.0, sv = 0.0, sa = 0.0;
    for (int j = pt; j < n; j += 8) {
        const int i = n0 + j;
        const double m = a.mass[i];
        const double Yx = (a.x[i] + a.ux[i]) - Cx, Yy = (a.y[i] + a.uy[i]) - Cy;
        const double dvx = (a.vx[i] - vcx) + om * Yy, dvy = (a.vy[i] - vcy) - om * Yx;
        const double dax = ((a.ax[i] - acx) + al * Yy) + om2 * Yx;
        const double day = ((a.ay[i] - acy) - al * Yx) + om2 * Yy;
        const double zx = (cp * Yx + sp * Yy) - c.tX[t0 + j], zy = (-sp * Yx + cp * Yy) - c.tY[t0 + j];
        const double bvx = cp * dvx + sp * dvy, bvy = -sp * dvx + cp * dvy;
        const double bax = cp * dax + sp * day, bay = -sp * dax + cp * day;
        const float fx = c.phi[((size_t)(t0 + j) * kClModes + k) * 2];
        const float fy = c.phi[((size_t)(t0 + j) * kClModes + k) * 2 + 1];
        sq += m * ((double)fx * zx + (double)fy * zy);
        sv += m * ((double)fx * bvx + (double)fy * bvy);
        sa += m * ((double)fx * bax + (double)fy * bay);
    }
    part[pt][k][0] = sq;
    part[pt][k][1] = sv;
    part[pt][k][2] = sa;
    __syncthreads();
    if (threadIdx.x < kClModes) {
        double q = 0.0, qv = 0.0, qa = 0.0;
        for (int u = 0; u < 8; ++u) {
            q += part[u][k][0];
            qv += part[u][k][1];
            qa += part[u][k][2];
        }
        c.qr[ci * kClModes + k] = q;
        c.qv[ci * kClModes + k] = qv;
        c.qa[ci * kClModes + k] = qa;
    }
}

// k_rc_sync: every node of every active reduced particle into the current
// nodal state
__global__ __launch_bounds__(256) void k_rc_sync(DevArgs a, ClArgs c) {
    __shared__ double Q[3][kClModes];
    const int ci = blockIdx.x;
    const int p = c.cpart[ci];
    if (!a.cl_on[p]) return;
    const int s = c.cshape[ci];
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    const int t0 = c.toff[s];
    if (threadIdx.x < kClModes) {
        Q[0][threadIdx.x] = c.qr[ci * kClModes + threadIdx.x];
        Q[1][threadIdx.x] = c.qv[ci * kClModes + threadIdx.x];
        Q[2][threadIdx.x] = c.qa[ci * kClModes + threadIdx.x];
    }
    __syncthreads();
    const RcRigid r = rc_rigid(c.rs + (size_t)ci * 16);
    int st = 0;
    for (int j = threadIdx.x; j < n; j += 256)
        st |= rc_write(a, c, n0 + j, t0 + j, r, Q[0], Q[1], Q[2], const_cast<double *>(a.ux),
                       const_cast<double *>(a.uy), const_cast<double *>(a.vx),
                       const_cast<double *>(a.vy), const_cast<double *>(a.ax),
                       const_cast<double *>(a.ay));
    if (st) atomicOr(a.status, st);
}

// k_rc_collect (at a list rebuild, after k_rc_mark): the active nodes of each
// reduced particle in ascending order (wavefront ballots), and the reduced
// positions the motion bound is measured from
__global__ __launch_bounds__(256) void k_rc_collect(DevArgs a, ClArgs c, const uint8_t *act) {
    __shared__ int wc[4];
    const int ci = blockIdx.x;
    const int p = c.cpart[ci];
    if (!a.cl_on[p]) return;
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int total = 0;
    for (int base = 0; base < n; base += 256) {
        const int j = base + (int)threadIdx.x;
        const bool f = j < n && act[n0 + j];
        const unsigned long long bal = __ballot(f);
        if (l == 0) wc[w] = __popcll(bal);
        __syncthreads();
        int off = total;
        for (int u = 0; u < w; ++u) off += wc[u];
        if (f) {
            const int rank = __popcll(bal & ((1ull << l) - 1ull));
            c.alist[(size_t)ci * c.max_n + off + rank] = n0 + j;
        }
        total += wc[0] + wc[1] + wc[2] + wc[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c.acnt[ci] = total;
        double *R = c.rs + (size_t)ci * 16;
        R[RS_RBX] = R[RS_CX];
        R[RS_RBY] = R[RS_CY];
        R[RS_RBPHI] = R[RS_PHI];
    }
    if (threadIdx.x < kClModes) c.qrb[ci * kClModes + threadIdx.x] = c.qr[ci * kClModes + threadIdx.x];
}

// ---------------------------------------------------------------------------
// periodic check against the plain bond force: per particle, the modal force
// of the closure vs the modal PD force (in c.gext after a mode-1 projection),
// and the largest true bond stretch (smax per node, from the force kernel)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cl_check_part(DevArgs a, ClArgs c, double err_tol,
                                                       double *per) {
    __shared__ double sh[4];
    const int ci = blockIdx.x;
    const int p = c.cpart[ci];
    double *out = per + (size_t)ci * 4;
    if (!a.cl_on[p]) {
        if (threadIdx.x == 0) out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    const int s = c.cshape[ci];
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    double mx = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) mx = fmax(mx, a.smax[n0 + k]);
    mx = block_max(mx, sh);
    if (threadIdx.x >= 64) return;
    const int k = threadIdx.x;
    double e2 = 0, n2 = 0, l2 = 0, q2 = 0;
    if (k < kClModes) {
        const double q = c.q[ci * kClModes + k];
        const double lq = -c.lam[s * kClModes + k] * q;
        const double gh = c.learned ? c.ghat[ci * kClModes + k] : lq;
        const double g = c.gext[ci * kClModes + k];
        e2 = (gh - g) * (gh - g);
        n2 = g * g;
        l2 = (lq - g) * (lq - g);
        q2 = lq * lq;
    }
    for (int o = 32; o > 0; o >>= 1) {
        e2 += __shfl_xor(e2, o, 64);
        n2 += __shfl_xor(n2, o, 64);
        l2 += __shfl_xor(l2, o, 64);
        q2 += __shfl_xor(q2, o, 64);
    }
    if (k == 0) {
        out[0] = e2;
        out[1] = n2;
        out[2] = l2;
        out[3] = 1.0;
        const double scale = fmax(sqrt(n2), sqrt(q2));
        if (mx > c.gate_frac * c.s0[s] || sqrt(e2) > err_tol * scale) {
            a.cl_on[p] = 0;
            list_particle_blocks(a, c, p);
            atomicAdd(c.fallbacks, 1ull);
        }
    }
}

// fixed-order sums of the per-particle check results: stats = [sum e2,
// sum n2, sum l2, checked particles]
__global__ __launch_bounds__(256) void k_cl_check_sum(const double *per, int Pc, double *stats) {
    __shared__ double sh[16];
    double v[4] = {0, 0, 0, 0};
    for (int ci = threadIdx.x; ci < Pc; ci += 256)
        for (int k = 0; k < 4; ++k) v[k] += per[(size_t)ci * 4 + k];
    block_sum<4>(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) stats[k] = v[k];
}

// ---------------------------------------------------------------------------
// the MLP forward (training, checks, snapshots): one workgroup of eight
// wavefronts per 16-row block.  The launch is latency-bound (2 000 rows are
// 125 workgroups), so the loads are issued at the start in the order they
// are needed, with no branch between them: the block's inputs, then every
// weight fragment and bias of the wave's three layers.  Every row of the
// block is computed and written, also those of particles that are off
// (their consumers skip them; rows are independent); a replay that has gone
// stale computes but writes nothing.
// ---------------------------------------------------------------------------
constexpr int kMlpWaves = 8;

__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp_fwd(MlpArgs m, DevArgs a, int list) {
    static_assert(16 * kClModes == 64 * kMlpWaves, "one input element per thread");
    __shared__ __align__(16) uint16_t Xs[16 * kXsStride];
    __shared__ __align__(16) uint16_t H1[16 * kHStride];
    __shared__ __align__(16) uint16_t H2[16 * kHStride];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rb = blockIdx.x;
    int s = m.shape, first = 16 * rb, cnt;
    if (m.rb_shape) {
        s = m.rb_shape[rb];
        first = m.rb_first[rb];
        cnt = m.rb_count[rb];
    } else {
        cnt = min(16, m.rows - first);
    }
    const int r = l & 15, kq = 4 * (l >> 4);
    // ---- this thread's input element (row, col) = (tid / 32, tid % 32) ---------
    // (indices clamped to the block's rows, so that no load waits on a branch)
    const int xrow = threadIdx.x / kClModes, xcol = threadIdx.x % kClModes;
    const int xr = min(xrow, cnt - 1);
    const double qin = m.q[(size_t)(m.idx ? m.idx[first + xr] : first + xr) * kClModes + xcol];
    const float sq = m.sig_q[s * kClModes + xcol];
    // ---- the wave's weights and biases --------------------------------------
    MlpWave<kMlpWaves> W;
    mlp_load<kMlpWaves>(W, m.wfr + (size_t)s * kClFrag, m.wf + (size_t)s * kClParams, wv, l);
    const bool last = wv < kClModes / 16;  // waves of the last layer
    const int n3 = 16 * (last ? wv : 0) + r;
    float sr3 = 0.0f;
    double lam3 = 0.0, q3[4] = {0.0, 0.0, 0.0, 0.0};
    if (last && m.g) {
        lam3 = m.lam[s * kClModes + n3];
        sr3 = m.sig_r[s * kClModes + n3];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = min(kq + t, cnt - 1);
            q3[t] = m.q[(size_t)(m.idx ? m.idx[first + row] : first + row) * kClModes + n3];
        }
    }
    // ---- inputs, bfloat16 -----------------------------------------------------
    {
        const float xv = xrow < cnt ? (float)(qin / (double)sq) : 0.0f;  // padding rows: 0
        const uint16_t b = f2bf(xv);
        Xs[xrow * kXsStride + xcol] = b;
        if (m.xb && xrow < cnt) m.xb[(size_t)(first + xrow) * kClModes + xcol] = b;
    }
    __syncthreads();
    mlp_hidden(Xs, kXsStride, W.w1, W.b1, H1, wv, l, first, cnt, m.z1, m.h1);
    __syncthreads();
    mlp_hidden(H1, kHStride, W.w2, W.b2, H2, wv, l, first, cnt, m.z2, m.h2);
    __syncthreads();
    if (last) {
        const bool stale = list && replay_stale(a, true);
        const f32x4 y = mlp_out<kMlpWaves>(H2, W, l);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = kq + t;
            if (stale || row >= cnt) continue;
            if (m.y) m.y[(size_t)(first + row) * kClModes + n3] = y[t];
            if (m.g)
                m.g[(size_t)(first + row) * kClModes + n3] = -lam3 * q3[t] + (double)sr3 * (double)y[t];
        }
    }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// C[M x N] = sum_k A[m][k] B[k][n], bfloat16 operands at arbitrary strides,
// float32 accumulation; one 16 x 16 tile per wavefront.
//   epi 0: C = acc
//   epi 1: C = acc * silu'(Z), and its bfloat16 copy in Cb (back-propagation
//          through a SiLU layer)
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t *A, long sam,
                                              long sak, const uint16_t *B, long sbk, long sbn,
                                              float *C, long ldc, int epi, const float *Z,
                                              uint16_t *Cb) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int tn = (N + 15) / 16, tm = (M + 15) / 16;
    const int tile = blockIdx.x * 4 + wv;
    if (tile >= tn * tm) return;
    const int m0 = 16 * (tile / tn), n0 = 16 * (tile % tn);
    const int r = l & 15, kq = 4 * (l >> 4), k8 = 8 * (l >> 4);
    const int am = m0 + r, bn = n0 + r;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        uint16_t av[8], bv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = k0 + k8 + t;
            av[t] = (am < M && k < K) ? A[(long)am * sam + (long)k * sak] : (uint16_t)0;
            bv[t] = (bn < N && k < K) ? B[(long)k * sbk + (long)bn * sbn] : (uint16_t)0;
        }
        acc = mfma32(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int mm = m0 + kq + t, nn = n0 + r;
        if (mm >= M || nn >= N) continue;
        float v = acc[t];
        if (epi == 1) {
            v *= dsilu_f(Z[(long)mm * ldc + nn]);
            Cb[(long)mm * ldc + nn] = f2bf(v);
        }
        C[(long)mm * ldc + nn] = v;
    }
}

// dy = 2 (y - r / sigma_r) / (rows * 32), r = g + lambda q of the batch's
// samples; each workgroup leaves its part of the squared error in part[]
__global__ __launch_bounds__(256) void k_mlp_loss(MlpArgs m, const double *g, float *dy,
                                                  uint16_t *dyb, double *part) {
    __shared__ double sh[4];
    const int s = m.shape;
    const int total = m.rows * kClModes;
    const float scale = 2.0f / (float)total;
    double acc[1] = {0.0};
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < total) {
        const int b = e / kClModes, k = e % kClModes;
        const int src = m.idx ? m.idx[b] : b;
        const double q = m.q[(size_t)src * kClModes + k];
        const double rr = g[(size_t)src * kClModes + k] + m.lam[s * kClModes + k] * q;
        const float t = (float)(rr / (double)m.sig_r[s * kClModes + k]);
        const float d = m.y[e] - t;
        const float v = scale * d;
        dy[e] = v;
        dyb[e] = f2bf(v);
        acc[0] = (double)d * (double)d;
    }
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// the mean squared error from the per-workgroup parts, in order
__global__ __launch_bounds__(256) void k_loss_sum(const double *part, int nparts, int total,
                                                  float *loss) {
    __shared__ double sh[4];
    double v[1] = {0.0};
    for (int k = threadIdx.x; k < nparts; k += 256) v[0] += part[k];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) *loss = (float)(v[0] / total);
}

// column sums of X [rows][cols] (bias gradients): one workgroup per column,
// a fixed-order reduction
__global__ __launch_bounds__(256) void k_colsum(const float *X, int rows, int cols, float *out) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < rows; b += 256) v[0] += (double)X[(size_t)b * cols + j];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) out[j] = (float)v[0];
}

__global__ void k_adam(float *w, uint16_t *wb, const float *g, float *mo, float *ve, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * mo[i] + (1.0f - b1) * gi;
    const float vi = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = mi;
    ve[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

// counter-based uniform in [0, 1): splitmix64 of (seed, index)
__device__ __forceinline__ double hash_u01(uint64_t seed, uint64_t i) {
    uint64_t z = seed + 0x9e3779b97f4a7c15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// W1, W2 uniform with variance 2 / (fan_in + fan_out); W3 and the biases
// zero, so the untrained closure is the linear one
// one shape's bfloat16 weights into fragment order (one element per thread)
__global__ __launch_bounds__(256) void k_mlp_pack(const uint16_t *wb, uint16_t *wfr) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= kClFrag) return;
    int off, K, f;
    if (o < kFragW2) {
        off = kOffW1, K = kClModes, f = (o - kFragW1) / kFragElems;
    } else if (o < kFragW3) {
        off = kOffW2, K = kClHidden, f = (o - kFragW2) / kFragElems;
    } else {
        off = kOffW3, K = kClHidden, f = (o - kFragW3) / kFragElems;
    }
    const int l = (o / 8) % 64, t = o % 8;
    const int tile = f / (K / 32), ks = f % (K / 32);
    const int n = 16 * tile + l % 16, k = 32 * ks + 8 * (l / 16) + t;
    wfr[o] = wb[off + n * K + k];
}

__global__ void k_mlp_init(float *w, uint16_t *wb, uint64_t seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kClParams) return;
    float v = 0.0f;
    if (i < kOffB1) {
        const double a = sqrt(6.0 / (kClModes + kClHidden));
        v = (float)(a * (2.0 * hash_u01(seed, (uint64_t)i) - 1.0));
    } else if (i >= kOffW2 && i < kOffB2) {
        const double a = sqrt(6.0 / (kClHidden + kClHidden));
        v = (float)(a * (2.0 * hash_u01(seed, (uint64_t)i) - 1.0));
    }
    w[i] = v;
    wb[i] = f2bf(v);
}

__global__ void k_batch_idx(int *idx, int rows, int64_t n, uint64_t seed, int64_t it) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= rows) return;
    const double u = hash_u01(seed ^ (0x5851f42d4c957f2dull * (uint64_t)(it + 1)), (uint64_t)b);
    int64_t k = (int64_t)(u * (double)n);
    idx[b] = (int)(k < n ? k : n - 1);
}

// sigma_q[k] = rms of q[:, k], sigma_r[k] = rms of (g + lambda q)[:, k]; 1 where zero
__global__ __launch_bounds__(256) void k_norm_stats(const double *q, const double *g,
                                                    const double *lam, int64_t n, float *sig_q,
                                                    float *sig_r) {
    __shared__ double sh[8];
    const int k = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double qq = q[j * kClModes + k];
        const double rr = g[j * kClModes + k] + lam[k] * qq;
        v[0] += qq * qq;
        v[1] += rr * rr;
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        const double a = sqrt(v[0] / (double)n), b = sqrt(v[1] / (double)n);
        sig_q[k] = a > 0.0 ? (float)a : 1.0f;
        sig_r[k] = b > 0.0 ? (float)b : 1.0f;
    }
}

__global__ void k_f32_to_bf16(const float *x, uint16_t *y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_cl_project(const DevArgs &a, const ClArgs &c, bool list, int mode, int max_n,
                             hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    // the buffers each mode reads
    if (mode == 0 ? !(a.cl_on && a.cl_fx && a.cl_fy) : !a.terms) return hipErrorInvalidValue;
    if (mode == 1 && !a.cl_on) return hipErrorInvalidValue;
    if (!c.rb_shape || c.n_rb <= 0) return hipErrorInvalidValue;
    if (!c.part || c.n_slices * kModalSlice < max_n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cl_moments, dim3(c.Pc), dim3(256), 0, s, a, c, list ? 1 : 0, mode);
    hipLaunchKernelGGL(k_cl_modal, dim3(c.n_rb, c.n_slices), dim3(512), 0, s, a, c, list ? 1 : 0,
                       mode);
    hipLaunchKernelGGL(k_cl_modal_sum, dim3((c.Pc + 7) / 8), dim3(256), 0, s, a, c, list ? 1 : 0,
                       mode);
    return hipGetLastError();
}

hipError_t launch_cl_apply(const DevArgs &a, const ClArgs &c, bool list, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!a.cl_on || !c.rb_shape) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cl_apply, dim3(c.n_rb, c.n_slices), dim3(512), 0, s, a, c, list ? 1 : 0);
    return hipGetLastError();
}

static bool rc_ready(const DevArgs &a, const ClArgs &c) {
    return a.cl_on && c.rs && c.qr && c.qv && c.qa && c.qrb && c.alist && c.acnt && c.Mt && c.I0 &&
           c.bvec && c.phimax && c.rmax;
}

hipError_t launch_rc_init(const DevArgs &a, const ClArgs &c, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!rc_ready(a, c)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rc_init, dim3(c.Pc), dim3(256), 0, s, a, c);
    return hipGetLastError();
}

hipError_t launch_rc_sync(const DevArgs &a, const ClArgs &c, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!rc_ready(a, c)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rc_sync, dim3(c.Pc), dim3(256), 0, s, a, c);
    return hipGetLastError();
}

hipError_t launch_rc_collect(const DevArgs &a, const ClArgs &c, const uint8_t *act, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!rc_ready(a, c) || !act) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rc_collect, dim3(c.Pc), dim3(256), 0, s, a, c, act);
    return hipGetLastError();
}

hipError_t launch_cl_check(const DevArgs &a, const ClArgs &c, double err_tol, double *per,
                           double *stats, hipStream_t s) {
    if (c.Pc <= 0) return hipSuccess;
    if (!a.cl_on || !a.smax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cl_check_part, dim3(c.Pc), dim3(256), 0, s, a, c, err_tol, per);
    hipLaunchKernelGGL(k_cl_check_sum, dim3(1), dim3(256), 0, s, per, c.Pc, stats);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpArgs &m, const DevArgs &a, bool list, hipStream_t s) {
    if (m.row_blocks <= 0) return hipSuccess;
    if (!m.wfr || !m.wf || !m.q) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(m.row_blocks), dim3(64 * kMlpWaves), 0, s, m, a, list ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(int M, int N, int K, const uint16_t *A, long sam, long sak,
                            const uint16_t *B, long sbk, long sbn, float *C, long ldc, int epi,
                            const float *Z, uint16_t *Cb, hipStream_t s) {
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm, dim3((tiles + 3) / 4), dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk,
                       sbn, C, ldc, epi, Z, Cb);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const MlpArgs &m, const double *g, float *dy, uint16_t *dyb, double *part,
                           float *loss, hipStream_t s) {
    const int total = m.rows * kClModes;
    const int nb = (total + 255) / 256;
    hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, s, m, g, dy, dyb, part);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, part, nb, total, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *X, int rows, int cols, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, s, X, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, uint16_t *wb, const float *g, float *m, float *v, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, wb, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const uint16_t *wb, uint16_t *wfr, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(kClFrag / 256), dim3(256), 0, s, wb, wfr);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *w, uint16_t *wb, uint64_t seed, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_init, dim3((kClParams + 255) / 256), dim3(256), 0, s, w, wb, seed);
    return hipGetLastError();
}

hipError_t launch_batch_idx(int *idx, int rows, int64_t n, uint64_t seed, int64_t it, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_idx, dim3((rows + 255) / 256), dim3(256), 0, s, idx, rows, n, seed, it);
    return hipGetLastError();
}

hipError_t launch_norm_stats(const double *q, const double *g, const double *lam, int64_t n,
                             float *sig_q, float *sig_r, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_stats, dim3(kClModes), dim3(256), 0, s, q, g, lam, n, sig_q, sig_r);
    return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((n + 255) / 256), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace pd
