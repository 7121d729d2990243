// pd_internal.h -- device data layout and kernel launch interface of libpd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/pd.h"

namespace pd {

constexpr uint32_t kBroken = 0x80000000u;  // broken bit of a bond slot
constexpr uint32_t kIndexMask = 0x7fffffffu;
constexpr int kSlice = 16;                  // SELL slice height: the nodes of one wavefront (4 lanes each)
constexpr int kBlLanes = 16;   // lanes per node of the candidate-list build
constexpr int kBlMaxc = 2048;  // longest candidate list (the build gathers it in LDS)
// nodes per workgroup of the plain-force-only pass (modal closure on), whatever
// the tuning (the unit of its workgroup list)
constexpr int kSelBlockNodes = 64;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 256;
constexpr int kSortItemsMax = 8;
// Keys per thread of a radix pass: one up to 64k keys (a workgroup of 256 keys
// each, one scatter round), more for larger sorts (at most kSortItemsMax), so
// that the per-digit scan over tiles stays short.
inline int sort_items(int N) {
    const int per = (N + 65535) / 65536;
    return per < 1 ? 1 : (per > kSortItemsMax ? kSortItemsMax : per);
}
inline int sort_tiles(int N) {
    const int tile = kSortBlock * sort_items(N);
    return (N + tile - 1) / tile;
}
// tiles of any sort of at most N keys (the hist buffer's size): up to 256 while
// the items grow, then those of N itself
inline int sort_tiles_max(int N) {
    const int t = sort_tiles(N);
    return t > 256 ? t : 256;
}
constexpr int kMaxLdsNodes = 1024;          // staged window limit (nodes)
constexpr int kWin = 6;                      // doubles per staged window node: x, y, ux, uy, V, pad
constexpr int kChunk = 64;                  // list-mode steps per graph replay
constexpr int kReplaysPerSync = 4;          // plain replays queued per host round trip

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
    double thr2;  // the reference-bond test |x_j - x_i|^2 < (eps - 1e-9 eps)^2
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
    int lanes;               // lanes per node of the list-mode step kernel (1, 2 or 4)
    // state: read buffers (cur) and write buffers (nxt)
    const double *ux, *uy, *vx, *vy, *ax, *ay;
    double *ux_o, *uy_o, *vx_o, *vy_o, *ax_o, *ay_o;
    // the displacement of the next position half-step, u + dt v + dt^2/2 a,
    // as the list-mode step kernel wrote it beside the state (unx_o) and the
    // next launch of the same replay reads it (unx) instead of evaluating it
    // from u, v and a for the node and every partner (closure off only)
    const double *unx, *uny;
    double *unx_o, *uny_o;
    // contact grid
    uint32_t *keys;       // [N] cell key per node
    const uint32_t *skey; // [N] sorted keys
    const int *perm;      // [N] sorted position -> node
    uint32_t *cell_start; // [ncells]
    uint32_t *cell_end;   // [ncells] one past the cell's last sorted entry
    double *spx, *spy;    // [N] positions in sorted order
    int *spart;           // [N] particle of sorted position
    const double *agg_gx0, *agg_gy0;  // grid origin per aggregate
    const int *agg_ncx, *agg_ncy;
    const uint32_t *agg_cell0;
    double cell, inv_cell;
    // walls
    const double *box;    // [A*4]
    const double *vtop;   // [A]
    // the pass of list-mode steps (tuning wall_pass, closure off): the nodes
    // within the list radius of a wall at the last rebuild and the wall force
    // the pass evaluates for each of them before the step kernel reads it;
    // the nodes with contact candidates and their contact sums
    int *wall_list;                  // [N]
    unsigned long long *wall_n;      // listed nodes
    double *wfx, *wfy;               // [N], valid at listed nodes
    int *cont_list;                  // [N] nodes with contact candidates
    unsigned long long *cont_n;      // listed nodes
    double *csum;                    // [N][4] their contact sums (self x, y; other x, y)
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
    uint32_t *brk_log;         // [N][4 lanes][4] partners of the bonds a step broke
    const uint8_t *row_full;   // [N] the row holds every same-particle node within eps
    uint8_t *node_broken;      // [N] one of the node's bonds is broken
    float *ubx, *uby;          // displacement at list build
    int maxc;                  // slots per node
    double Rl2;                // list radius squared, (R_c + skin)^2
    double move2;              // |u - u_build|^2 beyond which the list is stale
    unsigned long long *invalid_step;  // first step whose list is stale
    long long *step_base;      // steps completed before the current replay
    int chunk_k;               // index of this launch within the replay
    int *overflow;             // a node had more candidates than slots
    // modal closure: particles with cl_on[p] != 0 take their internal force
    // from the closure; the force kernel skips their bonds and leaves their
    // external (contact + wall) nodal force in cl_fx / cl_fy
    int *cl_on;                // [P] or null
    double *cl_fx, *cl_fy;     // [N]
    // M_FORCES: largest |stretch| over each node's intact bonds, or null
    double *smax;
    // with the closure on: the force workgroups holding nodes under the plain
    // force (a list that only grows), and its length
    const int *pd_blocks;
    const int *n_pd_blocks;
};

// ---- modal closure -----------------------------------------------------------
constexpr int kClModes = 32;        // modal amplitudes per particle (MLP width in and out)
constexpr int kClHidden = 256;      // hidden width
constexpr int kClMaxNodes = 1024;   // nodes per closure particle (projection LDS <= 64 KB)
constexpr int kClParams = kClHidden * kClModes + kClHidden + kClHidden * kClHidden + kClHidden +
                          kClModes * kClHidden + kClModes;
// packed parameter offsets: W1 [256][32], b1, W2 [256][256], b2, W3 [32][256], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kClHidden * kClModes;
constexpr int kOffW2 = kOffB1 + kClHidden;
constexpr int kOffB2 = kOffW2 + kClHidden * kClHidden;
constexpr int kOffW3 = kOffB2 + kClHidden;
constexpr int kOffB3 = kOffW3 + kClModes * kClHidden;
// The three weight matrices again, in matrix-core fragment order (what the
// MLP forward reads): fragment (tile, ks) of a [rows][K] matrix M is 64 lanes
// x 8 bfloat16, lane l holding M[16 tile + l % 16][32 ks + 8 (l / 16) + t],
// t = 0..7 (the B operand of v_mfma_f32_16x16x32_bf16 for the columns of the
// tile), so that one wavefront's operand load is 1 KB contiguous.
// W1 (16 x 1 fragments), W2 (16 x 8), W3 (2 x 8), back to back.
constexpr int kFragElems = 64 * 8;
constexpr int kFragW1 = 0;
constexpr int kFragW2 = kFragW1 + (kClHidden / 16) * (kClModes / 32) * kFragElems;
constexpr int kFragW3 = kFragW2 + (kClHidden / 16) * (kClHidden / 32) * kFragElems;
constexpr int kClFrag = kFragW3 + (kClModes / 16) * (kClHidden / 32) * kFragElems;
// per closure particle reduced quantities (red[16 * c + k])
enum { R_M = 0, R_CX, R_CY, R_VCX, R_VCY, R_PHI, R_I, R_OM, R_FX, R_FY, R_TAU, R_STRAIN, R_CONTACT,
       R_COS, R_SIN, R_ACTIVE, R_N };

// reduced state of a closure particle (reduced mode): centroid position,
// velocity and acceleration, rotation angle about the template orientation,
// angular velocity and acceleration; [Pc][16]
enum { RS_CX = 0, RS_CY, RS_VX, RS_VY, RS_AX, RS_AY, RS_PHI, RS_OM, RS_AL, RS_N,
       RS_RBX = 10, RS_RBY, RS_RBPHI };  // centroid and angle at the last list rebuild

struct ClArgs {
    int Pc;                    // closure particles (sorted by shape)
    const int *cpart;          // [Pc] particle index
    const int *cshape;         // [Pc] shape
    const int *poff;           // [P+1] first node of each particle
    const int *toff;           // [S] first template node of a shape
    const double *tX, *tY;     // template coordinates about the mass centroid
    const float *phi;          // modes: phi[(toff + i) * 64 + 2 k + c]
    const float2 *phiT;        // the same, mode-major: phiT[k * NT + toff + i] = (x, y)
    const int *rb_shape, *rb_first, *rb_count;  // blocks of <= 16 particles of one shape
    int n_rb;
    double *part;              // [Pc][n_slices][32][2] partial modal sums
    int n_slices;              // 32-node slices of the largest shape
    int NT;                    // template nodes of all shapes
    const double *lam;         // [S][32] eigenvalues (0 past the shape's mode count)
    const double *sig;         // [S][32] linear stretch of each mode, max over bonds
    const double *s0;          // [S] critical stretch of the shape's material
    const double *tau_c;       // [S] contact-load threshold of the gate
    double gate_frac;
    int learned;               // 0: g = -lambda q; 1: -lambda q + sigma_r MLP(q / sigma_q)
    double *red;               // [Pc][16]
    double *q, *gext, *ghat;   // [Pc][32]
    unsigned long long *fallbacks;
    // list of force workgroups with plain-force nodes, appended on fallback
    int *pd_blocks, *n_pd_blocks, *blk_listed;
    int block_nodes;
    // 1 in replays captured without the plain-force launch (no particle was
    // under the plain force at their start): a particle that leaves the
    // closure ends the replay after its step, so that the next replay has
    // that launch again
    int stop_on_fallback;
    // reduced mode: the particle's state is (centroid, angle, modal
    // amplitudes) and their rates; a step handles only the particle's active
    // nodes (listed at the last list rebuild: nodes with contact candidates,
    // candidates of others, or within the list radius of a wall), every node
    // is reconstructed before anything reads the nodal state
    double *rs;                // [Pc][16] RS_* entries
    double *qr, *qv, *qa;      // [Pc][32] modal amplitudes, rates, accelerations
    double *qrb;               // [Pc][32] modal amplitudes at the last list rebuild
    int *alist, *acnt;         // [Pc][max_n] active nodes (global index, ascending), [Pc] counts
    int max_n;                 // stride of alist
    const double *Mt, *I0, *bvec;  // [S] mass, polar moment of the template; [S][32] sum m X . phi_k
    const double *phimax, *rmax;   // [S][32] max_i |phi_k(i)|, [S] max_i |X_i|: the motion bound
};

// one forward pass of the MLP over `rows` rows of modal amplitudes
struct MlpArgs {
    int rows;
    int row_blocks;            // 16-row blocks
    const int *rb_shape;       // [row_blocks] or null (all rows shape `shape`)
    const int *rb_first;       // [row_blocks] first row or null (16 b)
    const int *rb_count;       // [row_blocks] rows in the block or null
    int shape;
    const int *idx;            // [rows] input row of each batch row, or null
    const double *q;           // inputs [*][32]
    const double *lam;         // [S][32]
    const uint16_t *wb;        // [S][kClParams] bfloat16 weights
    const uint16_t *wfr;       // [S][kClFrag] the same in fragment order
    const float *wf;           // [S][kClParams] float32 weights (biases read here)
    const float *sig_q, *sig_r;  // [S][32]
    double *g;                 // out: -lambda q + sigma_r y, [rows][32] (or null)
    // training caches (or null): inputs and activations of each layer
    float *y;                  // [rows][32]
    uint16_t *xb, *h1, *h2;    // [rows][32], [rows][256], [rows][256]
    float *z1, *z2;            // [rows][256]
};

struct ClState {
    bool ready = false;
    int mode = 0;              // 0 off, 1 linear, 2 learned
    int S = 0, Pc = 0;
    int check_every = 100;
    double err_tol = 0.05;
    std::vector<int> h_cpart, h_cshape, h_shape_n, h_toff, h_shape_first;
    std::vector<int> h_rb_shape, h_rb_first, h_rb_count;
    std::vector<int> h_nmodes;
    std::vector<int> h_trained;
    ClArgs ca{};
    MlpArgs ma{};
    // device buffers
    int *on = nullptr;
    double *lam = nullptr, *sig = nullptr, *s0 = nullptr, *tau_c = nullptr;
    float *phi = nullptr;
    float *phiT = nullptr;     // [32][NT] float2
    double *tX = nullptr, *tY = nullptr;
    uint16_t *wb = nullptr;
    uint16_t *wfr = nullptr;   // [S][kClFrag], repacked from wb after every change
    float *wf = nullptr, *sig_q = nullptr, *sig_r = nullptr;
    double *stats = nullptr;   // [4] device: sums of a check
    double *per = nullptr;     // [Pc][4] device: per-particle check results
    unsigned long long *fallbacks = nullptr;
    int max_n = 0;             // nodes of the largest closure shape
    // reduced mode
    bool reduced = false;
    bool plain_launch = true;  // the replays being enqueued include the plain-force launch
    double *rs = nullptr, *qr = nullptr, *qv = nullptr, *qa = nullptr, *qrb = nullptr;
    int *alist = nullptr, *acnt = nullptr;   // active nodes per closure particle
    uint8_t *act = nullptr;                  // [N] active flags (rebuild time)
    double *Mt = nullptr, *I0 = nullptr, *bvec = nullptr, *phimax = nullptr, *rmax = nullptr;
    std::vector<double> h_tX, h_tY;          // template coordinates (host copy)
    int64_t rb_step = 0;                     // step of the last list rebuild
    std::vector<std::vector<double>> h_phi;  // per shape [n_s][2][K] (float64)
    double last_err = -1.0, last_err_linear = -1.0;
    int64_t checks = 0;
    long long last_check_step = -1;
    // training workspace
    int tcap = 0;
    float *t_y = nullptr, *t_z1 = nullptr, *t_z2 = nullptr, *t_dy = nullptr, *t_dz2 = nullptr,
          *t_dz1 = nullptr, *t_grad = nullptr, *t_m = nullptr, *t_v = nullptr, *t_loss = nullptr;
    uint16_t *t_xb = nullptr, *t_h1 = nullptr, *t_h2 = nullptr, *t_dyb = nullptr,
             *t_dz2b = nullptr, *t_dz1b = nullptr;
    int *t_idx = nullptr;
    double *t_part = nullptr;  // [rows * 32 / 256 + 1] loss parts
    double *t_gbuf = nullptr;  // [rows][32] forward outputs
    std::vector<int64_t> adam_t;
    std::vector<double> h_lam, h_sig, h_tau_c;      // [S][32], [S][32], [S]
    std::vector<std::vector<std::pair<int, int>>> h_tbonds;  // template bonds, local indices
    double *fx = nullptr, *fy = nullptr, *smax = nullptr;
    int *pd_blocks = nullptr, *n_pd_blocks = nullptr, *blk_listed = nullptr;
    int blk_cap = 0;
    int64_t last_checked = 0;
};

struct Ctx {
    DevArgs a{};
    ClState cl;
    pd_tuning tune{64, 1.0, 1, 1, 1.0, 4, 0};
    bool list_valid = false;     // candidate lists match the current state
    int64_t rebuilds = 0;
    // steps between candidate-list rebuilds, running average (list mode): a
    // replay is made no longer than about this, so that a bed whose lists go
    // stale often does not queue launches that a stale step turns into no-ops
    double rebuild_interval = 1e9;
    int64_t last_rebuild_step = 0;
    // kChunk list-mode steps, [with the plain-force launch (closure on)][parity]
    hipGraphExec_t lgraph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    std::map<long, hipGraphExec_t> lgraph_n;          // shorter replays, by (parity, length)
    hipStream_t stream = nullptr;
    int device = 0;              // the HIP device current at setup
    bool own_stream = false;
    hipEvent_t caller_ev = nullptr;  // with an own stream: orders it after the legacy default stream
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
    // device control words of the list-mode steps, one block so that a round
    // of replays reads them back in one copy: first stale step, the steps
    // completed before the replay, status, and the longest candidate list of
    // a rebuild queued with the replay when it did not fit (else 0)
    struct Ctl {
        unsigned long long inv;
        long long base;
        int st;
        int over;
    } *ctl = nullptr;
    // pinned host copy of the control words, and the plain-force workgroup count
    struct Readback {
        Ctl ctl;
        int npb;
    } *rb = nullptr;
    double *U[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [buf][comp]
    double *UN[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}}; // next displacement, [buf][comp]
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
    std::vector<double> h_x, h_y, h_vol, h_mass;
    std::vector<double> h_box, h_vtop, h_agg_vol;  // per aggregate: box, top-wall speed, sum of V
    int *d_agg_pstart = nullptr, *d_agg_parts = nullptr;
    double *d_split = nullptr, *d_obs = nullptr, *d_pdamage = nullptr;
    int *d_cc = nullptr;  // fragments: labels [N], sizes [N], counts [P], flags [4]
    std::vector<int> h_poff, h_pmat;
    std::vector<MatConst> h_mc;
    const int *d_poff = nullptr;
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

// ---- host linear algebra (pd_eig.cpp) ----
// Eigenvalues (ascending, in w) and orthonormal eigenvectors (columns of A,
// row-major n x n, overwritten) of the symmetric matrix A.
void sym_eig(std::vector<double> &A, int n, std::vector<double> &w);

// ---- launch wrappers (pd_kernels.hip) ----
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_bonds_count(const BondArgs &b, int *rowlen, uint8_t *row_full, hipStream_t s);
hipError_t launch_node_broken(const DevArgs &a, hipStream_t s);
hipError_t launch_bonds_fill(const BondArgs &b, uint32_t *col, const uint32_t *slice_ptr,
                             hipStream_t s);
hipError_t launch_windows(const DevArgs &a, int *win_lo, int *win_hi, hipStream_t s);
hipError_t launch_keys(const DevArgs &a, int adv, uint32_t *hist, int G, hipStream_t s);
hipError_t launch_sort_pass(const uint32_t *kin, const int *vin, uint32_t *kout, int *vout, int N,
                            int shift, uint32_t *hist, uint32_t *dtotal, hipStream_t s,
                            hipEvent_t *ev, bool hist_done);
hipError_t launch_cells(const DevArgs &a, int adv, int advance_step, hipStream_t s);
int force_lds_cap(int max_win);
hipError_t launch_force(const DevArgs &a, int precision, int mode, int lds_cap, hipStream_t s,
                        bool list = false, int sel = 0, bool wall_pass = false);
// the pass of walls and contact candidates of list-mode steps: its node
// lists at a rebuild, then one launch before each step kernel
hipError_t launch_pass_mark(const DevArgs &a, hipStream_t s);
hipError_t launch_pass(const DevArgs &a, int precision, hipStream_t s);
hipError_t launch_cl_contact(const DevArgs &a, int precision, hipStream_t s);
// the reduced closure's step in one launch (contact, reduction, MLP when
// learned, update), one workgroup per block of <= 16 particles of one shape
hipError_t launch_rc_fused(const DevArgs &a, const ClArgs &c, const MlpArgs &m, int precision,
                           bool learned, bool list, hipStream_t s);
hipError_t launch_rc_mark(const DevArgs &a, uint8_t *act, double t_next, hipStream_t s);
hipError_t launch_observables(const DevArgs &a, double *split, const int *agg_pstart,
                              const int *agg_parts, const int *poff, double *out, hipStream_t s);
hipError_t launch_particle_damage(const DevArgs &a, const int *poff, double *out, hipStream_t s);
hipError_t launch_cc_init(int *L, int n, hipStream_t s);
hipError_t launch_cc_round(const DevArgs &a, int *L, int *changed, hipStream_t s);
hipError_t launch_cc_count(const DevArgs &a, const int *L, int *size, int min_nodes, int *count,
                           int *stats, hipStream_t s);
hipError_t launch_build_list(const DevArgs &a, hipStream_t s);
hipError_t launch_invalidate(const DevArgs &a, unsigned long long v, hipStream_t s);
hipError_t launch_arm_replay(const DevArgs &a, hipStream_t s);
hipError_t launch_round_start(const DevArgs &a, long long step, bool rebuild, hipStream_t s);
hipError_t launch_set_u64(unsigned long long *p, unsigned long long v, hipStream_t s);
hipError_t launch_sum_terms(const DevArgs &a, uint32_t mask, double *fx, double *fy, hipStream_t s);
hipError_t launch_damage(const DevArgs &a, double *phi, unsigned long long *nb, hipStream_t s);
hipError_t launch_contacts_count(const DevArgs &a, int *cnt, hipStream_t s);
hipError_t launch_cl_project(const DevArgs &a, const ClArgs &c, bool list, int mode, int max_n,
                             hipStream_t s);
hipError_t launch_cl_apply(const DevArgs &a, const ClArgs &c, bool list, hipStream_t s);
hipError_t launch_rc_init(const DevArgs &a, const ClArgs &c, hipStream_t s);
hipError_t launch_rc_sync(const DevArgs &a, const ClArgs &c, hipStream_t s);
hipError_t launch_rc_collect(const DevArgs &a, const ClArgs &c, const uint8_t *act, hipStream_t s);
hipError_t launch_cl_check(const DevArgs &a, const ClArgs &c, double err_tol, double *per,
                           double *stats, hipStream_t s);
hipError_t launch_mlp_forward(const MlpArgs &m, const DevArgs &a, bool list, hipStream_t s);
hipError_t launch_gemm_bf16(int M, int N, int K, const uint16_t *A, long sam, long sak,
                            const uint16_t *B, long sbk, long sbn, float *C, long ldc, int epi,
                            const float *Z, uint16_t *Cb, hipStream_t s);
hipError_t launch_mlp_loss(const MlpArgs &m, const double *g, float *dy, uint16_t *dyb,
                           double *part, float *loss, hipStream_t s);
hipError_t launch_colsum(const float *X, int rows, int cols, float *out, hipStream_t s);
hipError_t launch_adam(float *w, uint16_t *wb, const float *g, float *m, float *v, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_mlp_init(float *w, uint16_t *wb, uint64_t seed, hipStream_t s);
hipError_t launch_mlp_pack(const uint16_t *wb, uint16_t *wfr, hipStream_t s);
hipError_t launch_batch_idx(int *idx, int rows, int64_t n, uint64_t seed, int64_t it, hipStream_t s);
hipError_t launch_norm_stats(const double *q, const double *g, const double *lam, int64_t n,
                             float *sig_q, float *sig_r, hipStream_t s);
hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, int n, hipStream_t s);
hipError_t launch_contacts_fill(const DevArgs &a, const long long *off, int *pi, int *pj,
                                hipStream_t s);

}  // namespace pd
