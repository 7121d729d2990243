// pd_internal.h -- device data layout and kernel launch interface of libpd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pd.h"

namespace pd {

constexpr uint32_t kBroken = 0x80000000u;  // broken bit of a bond slot
constexpr uint32_t kIndexMask = 0x7fffffffu;
constexpr int kSlice = 16;                  // SELL slice height: the nodes of one wavefront (4 lanes each)
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kMaxLdsNodes = 1024;          // staged window limit (nodes)
constexpr int kChunk = 64;                  // list-mode steps per graph replay

// status bits raised by kernels
constexpr int kStEscaped = 1;
constexpr int kStNonfinite = 2;

// counters (int64, device)
enum { C_INTER = 0, C_SELF, C_STICK, C_SLIP, C_WALL, C_COINC, C_BROKEN, C_STEPS, C_N };

// kernel modes of the force kernel
enum { M_STEP = 0, M_FORCES = 1, M_PROLOGUE = 2 };

struct MatConst {
    double cw, s0, Kn, eps, rho, Kd_self;  // Kd_self = c_w / R_c
    int conic;
    int pad;
};

// Everything a kernel reads; passed by value.
struct DevArgs {
    int N, P, A, M;
    int n_slices;
    int radix_passes;
    // per node
    const double *x, *y, *vol, *mass;
    const int *part;      // node -> particle
    const int *pmat;      // particle -> material
    const int *pagg;      // particle -> aggregate
    const MatConst *mat;  // [M]
    // bonds (SELL-64)
    uint32_t *col;           // slots, j | broken
    const uint32_t *slice_ptr;  // [n_slices+1]
    const int *rowlen;       // [N]
    const int *win_lo, *win_hi;  // per force block
    int block_nodes;
    int use_lds;
    // state: read buffers (cur) and write buffers (nxt)
    const double *ux, *uy, *vx, *vy, *ax, *ay;
    double *ux_o, *uy_o, *vx_o, *vy_o, *ax_o, *ay_o;
    // contact grid
    uint32_t *keys;       // [N] cell key per node
    const uint32_t *skey; // [N] sorted keys
    const int *perm;      // [N] sorted position -> node
    uint32_t *cell_start; // [ncells]
    double *spx, *spy;    // [N] positions in sorted order
    int *spart;           // [N] particle of sorted position
    const double *agg_gx0, *agg_gy0;  // grid origin per aggregate
    const int *agg_ncx, *agg_ncy;
    const uint32_t *agg_cell0;
    double cell, inv_cell;
    // walls
    const double *box;    // [A*4]
    const double *vtop;   // [A]
    // scalars
    double Rc, Rc2, mu, rd, dt, hdt, hdt2, gx, gy;
    long long *step;      // device step counter (t = step * dt)
    int *status;
    unsigned long long *counters;
    int counting;
    // per-term outputs (M_FORCES): [5][2][N]
    double *terms;
    // contact candidate lists (pairs within the list radius at build time,
    // intact bonds excluded), slot k of node i at clist[k * N + i]
    uint32_t *clist;
    int *clist_n;
    float *ubx, *uby;          // displacement at list build
    int maxc;                  // slots per node
    double Rl2;                // list radius squared, (R_c + skin)^2
    double move2;              // |u - u_build|^2 beyond which the list is stale
    unsigned long long *invalid_step;  // first step whose list is stale
    long long *step_base;      // steps completed before the current replay
    int chunk_k;               // index of this launch within the replay
    int *overflow;             // a node had more candidates than slots
};

struct Ctx {
    DevArgs a{};
    pd_tuning tune{64, 1.0, 1, 1, 1.0};
    bool list_valid = false;     // candidate lists match the current state
    int64_t rebuilds = 0;
    hipGraphExec_t lgraph[2] = {nullptr, nullptr};  // kChunk list-mode steps per parity
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = 0;
    int cur = 0;                 // index of the buffer with the current state
    long long step = 0;          // host copy of the step counter
    int status = 0;              // sticky status
    int64_t nnz = 0, nslots = 0;
    int64_t ncells = 0;
    int max_win = 0;
    std::string err;
    // owned device buffers
    std::vector<void *> owned;
    double *U[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buf][comp]
    double *V[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    double *Acc[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    uint32_t *keys_alt = nullptr;
    int *perm_alt = nullptr;
    uint32_t *skey_buf = nullptr;
    int *perm_buf = nullptr;
    uint32_t *hist = nullptr;     // [kRadix * max_tiles]
    uint32_t *dtotal = nullptr;   // [kRadix] per pass
    int *win_lo = nullptr, *win_hi = nullptr;
    int *dev_i = nullptr;         // scratch ints
    double *dev_d = nullptr;      // scratch doubles
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // two steps starting at cur = 0 / 1
    bool graph_valid = false;
    int counting = 0;
    // host-side copies needed by setup/validation
    int N = 0, P = 0, A = 0, M = 0;
    std::vector<int> h_rowlen;
    std::vector<uint32_t> h_slice_ptr;
    // per-aggregate grid (host)
    std::vector<double> h_gx0, h_gy0;
    std::vector<int> h_ncx, h_ncy;
    std::vector<uint32_t> h_cell0;
};

// arguments of the reference-bond build
struct BondArgs {
    const double *x, *y;
    const int *part, *pmat, *poff;
    const double *seg;   // barrier segments (ax, ay, bx, by), world frame
    const int *seg_off;  // [P+1]
    const double *thr2;  // [M] (eps - 1e-9 eps)^2
    int N;
};

// ---- launch wrappers (pd_kernels.hip) ----
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_bonds_count(const BondArgs &b, int *rowlen, hipStream_t s);
hipError_t launch_bonds_fill(const BondArgs &b, uint32_t *col, const uint32_t *slice_ptr,
                             hipStream_t s);
hipError_t launch_windows(const DevArgs &a, int *win_lo, int *win_hi, hipStream_t s);
hipError_t launch_keys(const DevArgs &a, int adv, hipStream_t s);
hipError_t launch_sort_pass(const uint32_t *kin, const int *vin, uint32_t *kout, int *vout, int N,
                            int shift, uint32_t *hist, uint32_t *dtotal, hipStream_t s,
                            hipEvent_t *ev);
hipError_t launch_cells(const DevArgs &a, int adv, int advance_step, hipStream_t s);
int force_lds_cap(int max_win);
hipError_t launch_force(const DevArgs &a, int precision, int mode, int lds_cap, hipStream_t s,
                        bool list = false);
hipError_t launch_build_list(const DevArgs &a, hipStream_t s);
hipError_t launch_invalidate(const DevArgs &a, unsigned long long v, hipStream_t s);
hipError_t launch_set_u64(unsigned long long *p, unsigned long long v, hipStream_t s);
hipError_t launch_sum_terms(const DevArgs &a, uint32_t mask, double *fx, double *fy, hipStream_t s);
hipError_t launch_damage(const DevArgs &a, double *phi, unsigned long long *nb, hipStream_t s);
hipError_t launch_contacts_count(const DevArgs &a, int *cnt, hipStream_t s);
hipError_t launch_contacts_fill(const DevArgs &a, const long long *off, int *pi, int *pj,
                                hipStream_t s);

}  // namespace pd
