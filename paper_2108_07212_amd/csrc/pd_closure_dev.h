// pd_closure_dev.h -- device code shared by the closure kernels and the
// step kernel of the reduced closure (which also evaluates contact): fixed-order
// workgroup sums, the replay rule, fallback bookkeeping, and the reduced
// form's reconstruction of nodes from the rigid + modal state.
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

}  // namespace pd
