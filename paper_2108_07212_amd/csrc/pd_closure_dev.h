// pd_closure_dev.h -- device code shared by the closure kernels and the
// step kernel of the reduced closure (which also evaluates contact): fixed-order
// workgroup sums, the replay rule, fallback bookkeeping, and the reduced
// form's reconstruction, reduction and update.
#pragma once

#include "pd_internal.h"

namespace pd {

// sums of NV doubles over a 256-thread workgroup, in a fixed order (wave
// butterflies, then the four waves in order); every thread gets the sums
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *sh) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((sh[k] + sh[NV + k]) + sh[2 * NV + k]) + sh[3 * NV + k];
}

// a particle that leaves the closure: list the force workgroups holding its
// nodes (each at most once) for the plain-force launch of the next step; in a
// replay without that launch, end the replay after this step (list mode)
__device__ void list_particle_blocks(const DevArgs &a, const ClArgs &c, int p) {
    const int n0 = c.poff[p], n1 = c.poff[p + 1];
    for (int b = n0 / c.block_nodes; b <= (n1 - 1) / c.block_nodes; ++b)
        if (atomicExch(&c.blk_listed[b], 1) == 0) c.pd_blocks[atomicAdd(c.n_pd_blocks, 1)] = b;
    if (c.stop_on_fallback) {
        const long long sprev = *a.step_base + a.chunk_k;
        atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));
    }
}

// list mode: a launch past the first stale step of a replay does nothing (the
// same rule as the force kernel)
__device__ __forceinline__ bool replay_stale(const DevArgs &a, bool list) {
    if (!list) return false;
    const long long sprev = *a.step_base + a.chunk_k;
    return (unsigned long long)(sprev + 1) >= *a.invalid_step;
}

struct RcRigid {
    double cx, cy, vx, vy, ax, ay, cp, sp, om, al;
};

__device__ __forceinline__ RcRigid rc_rigid(const double *R) {
    RcRigid r;
    r.cx = R[RS_CX];
    r.cy = R[RS_CY];
    r.vx = R[RS_VX];
    r.vy = R[RS_VY];
    r.ax = R[RS_AX];
    r.ay = R[RS_AY];
    r.cp = cos(R[RS_PHI]);
    r.sp = sin(R[RS_PHI]);
    r.om = R[RS_OM];
    r.al = R[RS_AL];
    return r;
}

// body-frame position X + Phi q, modal velocity Phi qv and acceleration
// Phi qa of template node t (Q, Qv, Qa in LDS; pass null to skip)
__device__ __forceinline__ void rc_body(const ClArgs &c, int t, const double *Q, const double *Qv,
                                        const double *Qa, double &zx, double &zy, double &wx,
                                        double &wy, double &bx, double &by) {
    const float4 *row = reinterpret_cast<const float4 *>(c.phi + (size_t)t * 2 * kClModes);
    zx = c.tX[t];
    zy = c.tY[t];
    wx = wy = bx = by = 0.0;
#pragma unroll 4
    for (int k2 = 0; k2 < kClModes / 2; ++k2) {
        const float4 f = row[k2];  // (x, y) of modes 2 k2 and 2 k2 + 1
        const int k = 2 * k2;
        zx += (double)f.x * Q[k] + (double)f.z * Q[k + 1];
        zy += (double)f.y * Q[k] + (double)f.w * Q[k + 1];
        if (Qv) {
            wx += (double)f.x * Qv[k] + (double)f.z * Qv[k + 1];
            wy += (double)f.y * Qv[k] + (double)f.w * Qv[k + 1];
        }
        if (Qa) {
            bx += (double)f.x * Qa[k] + (double)f.z * Qa[k + 1];
            by += (double)f.y * Qa[k] + (double)f.w * Qa[k + 1];
        }
    }
}

// node i (template node t) of a reduced particle into the given buffers
__device__ __forceinline__ int rc_write(const DevArgs &a, const ClArgs &c, int i, int t,
                                        const RcRigid &r, const double *Q, const double *Qv,
                                        const double *Qa, double *ux, double *uy, double *vx,
                                        double *vy, double *ax, double *ay) {
    double zx, zy, wx, wy, bx, by;
    rc_body(c, t, Q, Qv, Qa, zx, zy, wx, wy, bx, by);
    const double Yx = r.cp * zx - r.sp * zy, Yy = r.sp * zx + r.cp * zy;
    const double px = r.cx + Yx, py = r.cy + Yy;
    const double om2 = r.om * r.om;
    const double nvx = (r.vx - r.om * Yy) + (r.cp * wx - r.sp * wy);
    const double nvy = (r.vy + r.om * Yx) + (r.sp * wx + r.cp * wy);
    const double nax = ((r.ax - r.al * Yy) - om2 * Yx) + (r.cp * bx - r.sp * by);
    const double nay = ((r.ay + r.al * Yx) - om2 * Yy) + (r.sp * bx + r.cp * by);
    ux[i] = px - a.x[i];
    uy[i] = py - a.y[i];
    vx[i] = nvx;
    vy[i] = nvy;
    ax[i] = nax;
    ay[i] = nay;
    return (isfinite(px) && isfinite(py) && isfinite(nvx) && isfinite(nvy)) ? 0 : kStNonfinite;
}

// rc_reduce_body (a step of closure particle ci, one workgroup, after the
// contact forces of its active nodes): positions of the reduced state advanced, then the external nodal forces
// (contact and walls act only on active nodes) reduced to the total force,
// the torque about the centroid (arms from the advanced nodal positions the
// contact forces were evaluated at), the contact load and the modal force
// Phi^T R(-phi) f; q goes to the MLP's input
__device__ __forceinline__ void rc_reduce_body(const DevArgs &a, const ClArgs &c, int list, int ci) {
    __shared__ double red[4 * 4];
    __shared__ double FB[2][kClMaxNodes];
    __shared__ double Q[kClModes];
    __shared__ double part[8][kClModes];
    __shared__ double Rg[3];
    if (replay_stale(a, list)) return;
    const int p = c.cpart[ci];
    double *RR = c.red + (size_t)ci * 16;
    if (!a.cl_on[p]) {
        if (threadIdx.x == 0) RR[R_ACTIVE] = 0.0;
        return;
    }
    const int s = c.cshape[ci];
    const int n0 = c.poff[p];
    const int t0 = c.toff[s];
    const int na = c.acnt[ci];
    const int *al = c.alist + (size_t)ci * c.max_n;
    double *R = c.rs + (size_t)ci * 16;
    const int tid = threadIdx.x;
    if (tid < kClModes) {
        const int k = tid;
        const double q = (c.qr[ci * kClModes + k] + a.dt * c.qv[ci * kClModes + k]) +
                         a.hdt2 * c.qa[ci * kClModes + k];
        Q[k] = q;
        c.qr[ci * kClModes + k] = q;
        c.q[ci * kClModes + k] = q;
    } else if (tid == kClModes) {
        const double cx = (R[RS_CX] + a.dt * R[RS_VX]) + a.hdt2 * R[RS_AX];
        const double cy = (R[RS_CY] + a.dt * R[RS_VY]) + a.hdt2 * R[RS_AY];
        const double phi = (R[RS_PHI] + a.dt * R[RS_OM]) + a.hdt2 * R[RS_AL];
        R[RS_CX] = cx;
        R[RS_CY] = cy;
        R[RS_PHI] = phi;
        Rg[0] = cx;
        Rg[1] = cy;
        Rg[2] = phi;
    }
    __syncthreads();
    const double cp = cos(Rg[2]), sp = sin(Rg[2]);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < na; b += 256) {
        const int i = al[b];
        const double fx = a.cl_fx[i], fy = a.cl_fy[i];
        const double Yx = (a.x[i] + a.ux_o[i]) - Rg[0], Yy = (a.y[i] + a.uy_o[i]) - Rg[1];
        v[0] += fx;
        v[1] += fy;
        v[2] += Yx * fy - Yy * fx;
        v[3] += sqrt(fx * fx + fy * fy);
        FB[0][b] = cp * fx + sp * fy;
        FB[1][b] = -sp * fx + cp * fy;
    }
    block_sum<4>(v, red);  // (syncs, so FB is complete afterwards)
    const int k = tid & 31, pt = tid >> 5;
    double g = 0.0;
    for (int b = pt; b < na; b += 8) {
        const int t = t0 + (al[b] - n0);
        const float fx = c.phi[((size_t)t * kClModes + k) * 2];
        const float fy = c.phi[((size_t)t * kClModes + k) * 2 + 1];
        g += (double)fx * FB[0][b] + (double)fy * FB[1][b];
    }
    part[pt][k] = g;
    __syncthreads();
    if (tid < 64) {  // wavefront 0: lanes 0..31 hold the modes
        double ge = 0.0, sb = 0.0, bq = 0.0;
        if (tid < kClModes) {
            for (int u = 0; u < 8; ++u) ge += part[u][k];
            c.gext[ci * kClModes + k] = ge;
            const double q = Q[k];
            sb = fabs(q) * c.sig[s * kClModes + k];
            bq = 2.0 * c.bvec[s * kClModes + k] * q + q * q;
        }
        for (int o = 16; o > 0; o >>= 1) {
            sb += __shfl_xor(sb, o, 64);
            bq += __shfl_xor(bq, o, 64);
        }
        if (tid == 0) {
            RR[R_M] = c.Mt[s];
            RR[R_CX] = Rg[0];
            RR[R_CY] = Rg[1];
            RR[R_PHI] = Rg[2];
            RR[R_COS] = cp;
            RR[R_SIN] = sp;
            RR[R_I] = c.I0[s] + bq;
            RR[R_FX] = v[0];
            RR[R_FY] = v[1];
            RR[R_TAU] = v[2];
            RR[R_CONTACT] = v[3];
            RR[R_STRAIN] = sb;
            RR[R_ACTIVE] = 1.0;
        }
    }
}

// rc_update_body (the end of a step of closure particle ci, one workgroup):
// accelerations and rates of the reduced
// state (F/M + g, tau/I, the closure's modal force plus the external one),
// the gate, the reconstruction of the active nodes (every node of a particle
// that leaves the closure) into the step's output state, and the bound on
// every node's motion since the last list rebuild (the particle's next
// position against its rebuild one, through centroid, angle and modes)
__device__ __forceinline__ void rc_update_body(const DevArgs &a, const ClArgs &c, int list, int ci) {
    __shared__ double Q[3][kClModes];
    __shared__ double Rn[16];
    __shared__ int fb;
    if (replay_stale(a, list)) return;
    const double *RR = c.red + (size_t)ci * 16;
    if (RR[R_ACTIVE] == 0.0) return;
    const int p = c.cpart[ci];
    const int s = c.cshape[ci];
    const int n0 = c.poff[p], n = c.poff[p + 1] - n0;
    const int t0 = c.toff[s];
    const int na = c.acnt[ci];
    const int *al = c.alist + (size_t)ci * c.max_n;
    double *R = c.rs + (size_t)ci * 16;
    const int tid = threadIdx.x;
    __shared__ double mb[2];
    if (tid < kClModes) {
        const int k = tid;
        const double q = c.qr[ci * kClModes + k];
        const double g = c.learned ? c.ghat[ci * kClModes + k] : -c.lam[s * kClModes + k] * q;
        const double qa = g + c.gext[ci * kClModes + k];
        const double qv = c.qv[ci * kClModes + k] + a.hdt * (c.qa[ci * kClModes + k] + qa);
        c.qv[ci * kClModes + k] = qv;
        c.qa[ci * kClModes + k] = qa;
        Q[0][k] = q;
        Q[1][k] = qv;
        Q[2][k] = qa;
        // the modal part of the motion bound, at the next step's amplitudes
        const double pm = c.phimax[s * kClModes + k];
        const double qb = c.qrb[ci * kClModes + k];
        double dq = fabs(((q + a.dt * qv) + a.hdt2 * qa) - qb) * pm;
        double zq = fabs(qb) * pm;
        for (int o = 16; o > 0; o >>= 1) {
            dq += __shfl_xor(dq, o, 32);
            zq += __shfl_xor(zq, o, 32);
        }
        if (k == 0) {
            mb[0] = dq;
            mb[1] = zq;
        }
    } else if (tid == kClModes) {
        const double M = RR[R_M];
        const double ax = RR[R_FX] / M + a.gx, ay = RR[R_FY] / M + a.gy;
        const double al = RR[R_TAU] / RR[R_I];
        const double vx = R[RS_VX] + a.hdt * (R[RS_AX] + ax);
        const double vy = R[RS_VY] + a.hdt * (R[RS_AY] + ay);
        const double om = R[RS_OM] + a.hdt * (R[RS_AL] + al);
        R[RS_VX] = vx;
        R[RS_VY] = vy;
        R[RS_AX] = ax;
        R[RS_AY] = ay;
        R[RS_OM] = om;
        R[RS_AL] = al;
        for (int u = 0; u < RS_N; ++u) Rn[u] = R[u];
        // gate for the next step: past gate_frac s0 on the stretch bound, or
        // past tau_c on the contact load, the particle leaves the closure
        // with every node reconstructed now
        int off = 0;
        if (RR[R_STRAIN] > c.gate_frac * c.s0[s] || RR[R_CONTACT] > c.tau_c[s]) {
            off = 1;
            a.cl_on[p] = 0;
            list_particle_blocks(a, c, p);
            atomicAdd(c.fallbacks, 1ull);
        }
        fb = off;
    }
    __syncthreads();
    const RcRigid r = rc_rigid(Rn);
    const int cnt = fb ? n : na;
    int st = 0, stale = 0;
    for (int b = tid; b < cnt; b += 256) {
        const int i = fb ? n0 + b : al[b];
        st |= rc_write(a, c, i, t0 + (i - n0), r, Q[0], Q[1], Q[2], a.ux_o, a.uy_o, a.vx_o,
                       a.vy_o, a.ax_o, a.ay_o);
        if (list && fb) {  // a particle leaving the closure: its nodes' own check
            const double unx = (a.ux_o[i] + a.dt * a.vx_o[i]) + a.hdt2 * a.ax_o[i];
            const double uny = (a.uy_o[i] + a.dt * a.vy_o[i]) + a.hdt2 * a.ay_o[i];
            const double ex = unx - (double)a.ubx[i], ey = uny - (double)a.uby[i];
            if (!(ex * ex + ey * ey <= a.move2)) stale = 1;
        }
    }
    if (list && !fb && tid == 0) {
        // |c' - c_rb| + |phi' - phi_rb| (r_max + sum |q_rb| phimax) + sum |q' - q_rb| phimax
        // bounds every node's displacement since the rebuild, at the next step
        const double cx = (Rn[RS_CX] + a.dt * Rn[RS_VX]) + a.hdt2 * Rn[RS_AX];
        const double cy = (Rn[RS_CY] + a.dt * Rn[RS_VY]) + a.hdt2 * Rn[RS_AY];
        const double ph = (Rn[RS_PHI] + a.dt * Rn[RS_OM]) + a.hdt2 * Rn[RS_AL];
        const double B = hypot(cx - R[RS_RBX], cy - R[RS_RBY]) +
                         fabs(ph - R[RS_RBPHI]) * (c.rmax[s] + mb[1]) + mb[0];
        if (!(B * B <= a.move2)) stale = 1;
    }
    if (st) atomicOr(a.status, st);
    if (__syncthreads_or(stale) && tid == 0) {
        const long long sprev = *a.step_base + a.chunk_k;
        atomicMin(a.invalid_step, (unsigned long long)(sprev + 2));
    }
}

}  // namespace pd
