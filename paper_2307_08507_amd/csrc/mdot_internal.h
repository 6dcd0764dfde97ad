// Internal layout shared by the host orchestration (mdot_api.cpp) and the kernels
// (mdot_kernels.hip). Not part of the public ABI.
#pragma once
#include <stdint.h>

#include "../../include/mdot.h"

namespace mdot {

// Tile geometry of the fused sweep: a workgroup of 4 wave64s covers BR rows x BC columns;
// each lane owns 4 consecutive columns, each wave RPW consecutive rows.
constexpr int kWG = 256;
constexpr int kBC = 256;
constexpr int kRPW = 16;
constexpr int kBR = 4 * kRPW;
constexpr int kVecWG = 256;

// Finalize kernel geometry: the tile partials of each entry of the (m + n)-vectors (rows, then
// columns) are combined by a group of L lanes (a power of two, at most 64) that each fold up to
// fin_per(m, n) of them. Rows and columns have their own L: a row combines one partial per column
// tile, a column one per row tile (4 times as many on a square problem), so a row needs fewer
// lanes. The row groups fill the first fin_vblocks_r(m, n) virtual workgroups, the column groups
// the rest, fin_vblocks(m, n) in all, run on fin_grid(m, n) workgroups. Depends on the sizes
// only, so the summation order of every entry is fixed by them. Past 8192 rows or columns each
// lane takes 32 partials, so that the groups fit in kFinMaxGrid workgroups without a second round
// (n = 16384: 2 lanes per row, 8 per column, 640 workgroups; with 8 per lane it would be 32 lanes
// per column and several rounds). Past 256 row tiles (more than 16384 rows) the column groups
// have kFinLanesLarge lanes, each folding its share of the partials in batches of 32 loads: the 8
// entries of a wave then read 8 consecutive partials of each row tile, so a load instruction
// touches 8 cache lines instead of one line per lane (L = 64 at 1561 row tiles); the row groups
// there take as many lanes as 32 partials each need, at most kFinLanesLarge.
constexpr int kFinMaxGrid = 1024;
constexpr int kFinLanesLarge = 8;
constexpr int fin_per(int m, int n) { return (m > n ? m : n) > 8192 ? 32 : 8; }
// the fewest lanes (a power of two, at most 64) that fold q partials at `per` each
constexpr int fin_lanes_for(int q, int per)
{
    int L = 1;
    while (L < 64 && L * per < q) L <<= 1;
    return L;
}
constexpr int fin_large(int m) { return (m + kBR - 1) / kBR > 256; }
constexpr int fin_lanes_r(int m, int n)
{
    const int nct = (n + kBC - 1) / kBC;
    if (fin_large(m)) {
        const int L = fin_lanes_for(nct, 32);
        return L < kFinLanesLarge ? L : kFinLanesLarge;
    }
    return fin_lanes_for(nct, fin_per(m, n));
}
constexpr int fin_lanes_c(int m, int n)
{
    return fin_large(m) ? kFinLanesLarge : fin_lanes_for((m + kBR - 1) / kBR, fin_per(m, n));
}
constexpr int fin_vblocks_r(int m, int n) { return (m * fin_lanes_r(m, n) + kVecWG - 1) / kVecWG; }
constexpr int fin_vblocks(int m, int n) { return fin_vblocks_r(m, n) + (n * fin_lanes_c(m, n) + kVecWG - 1) / kVecWG; }
constexpr int fin_grid(int m, int n) { return fin_vblocks(m, n) < kFinMaxGrid ? fin_vblocks(m, n) : kFinMaxGrid; }
// Finalize kernel instances, each with the registers its sizes need: kFinSmall for at most 8192
// rows and columns (fin_per = 8), kFinMid for larger problems of at most 256 row tiles, kFinAll
// for any size. A batch takes the largest instance one of its problems needs; every instance
// computes the same bits for the sizes it takes.
constexpr int kFinSmall = 0, kFinMid = 1, kFinAll = 2;
constexpr int fin_instance(int fin_per, int nrt) { return fin_per == 8 ? kFinSmall : (nrt <= 256 ? kFinMid : kFinAll); }

// What the next sweep does.
enum SweepMode : int32_t { SM_NONE = 0, SM_LSE = 1, SM_R1 = 2, SM_R2 = 3, SM_MAX = 4 };
// Phase of an LSE sweep.
enum LsPhase : int32_t { LS_INIT = 0, LS_TRIAL = 1, LS_FORCE = 2, LS_STANDALONE = 3 };
// O(n) work the vector kernel applies before the next sweep (bit mask, applied in this order).
enum VecAction : int32_t { VA_ACCEPT = 1, VA_SAVE_BEST = 2, VA_STAGE_INIT = 4, VA_ROUND_PREP = 8 };
// How an accepted step forms the next direction (State::reset, bit mask). RS_RESET: p = d,
// else p = d + beta p. d is the Sinkhorn direction s, or the diagonal-Hessian direction s~
// (stored by the finalize kernel of the trial) with RS_TILDE. RS_ROWS / RS_COLS keep only the
// row or column entries of d (the Sinkhorn projector's half-steps).
enum ResetBits : int32_t { RS_RESET = 1, RS_TILDE = 2, RS_ROWS = 4, RS_COLS = 8 };
// The line-search phase of the Sinkhorn projector's half-steps (alpha = 1, always accepted).
constexpr int32_t LS_SINK = 4;
constexpr double kOutrUnit = 1048576.0;  // 2^20: D_BAD's unit for out-of-range ratios

// Per-block partial reductions written by the row / column finalizers.
enum Dot : int {
    // LSE sweep (trial values at alpha; y = g_new - g_cur)
    D_PHI = 0,   // <p, g_new>            = phi'(alpha)            (App. B, eq. (phiprime))
    D_NUM = 1,   // <y, -s_new>           numerator of beta        (eq. (beta_PPR_OT))
    D_DEN = 2,   // <y, p>                denominator of beta
    D_SG = 3,    // <s_new, g_new>
    D_GN = 4,    // ||g_new||_1
    D_BAD = 5,   // number of rows/columns outside the exponent range, plus 2^20 times the
                 // number of ratios r~/r(P), c~/c(P) outside [0.01, 100] (precond variant)
    D_GNR = 6,   // ||g_new||_1 over the rows alone (Sinkhorn projector)
    D_NUMT = 6,  // <y, -s~_new>  numerator of beta with the diagonal-Hessian direction (precond)
    D_SGT = 7,   // <s~_new, g_new> (precond)
    // R1 sweep
    D_CG1 = 0,   // sum_j c_j g'_j   (from f = u/gamma)
    D_CG2 = 1,   // sum_j c_j g'_j   (from the finite-difference potentials)
    D_RF1 = 2,   // sum_i r_i f''_i  (from g = v/gamma)
    D_RF2 = 3,   // sum_i r_i f''_i  (finite difference)
    D_ERRC = 4,  // sum_j err_c_j
    // R2 sweep
    D_A = 0,     // sum_ij F'_ij C_ij
    D_ERRR = 1,  // sum_i err_r_i  (= ||err_r||_1, err_r >= 0)
    D_EC = 2,    // sum_i err_r_i (C err_c)_i
    D_RFP1 = 3,  // sum_i r_i f'_i
    D_RFP2 = 4,
    D_CGP1 = 5,  // sum_j c_j g''_j
    D_CGP2 = 6,
    // max pass
    kNDot = 8
};

struct DevParams {
    double p, q, gamma_i, gamma_f, target, c1, c2, hmin;
    double tol_floor;     // lower limit of the PNCG tolerance eps_d / 2
    double f32_min_tol;   // F32 sweeps while eps_d / 2 >= this, FP64 exp below it (initial floor)
    double mix_gamma;     // MIXED: stages with gamma <= this run on the FP16 copy (0: none)
    double hterm;         // entropy term of eps_d = hterm / gamma^p: H_min, or log n (App. C)
    double w_fixed;       // fixed smoothing weight (App. D), used when smooth_fixed
    int64_t max_sweeps;
    int32_t max_ls_trials, max_pncg_iters;
    int32_t adaptive, exp64_default, warm_start, n;
    int32_t projector, precond, smooth_fixed, pad_;
};

// Scalar solver state in device memory. Written only by the last workgroup of a sweep
// (one thread), read by every thread of the next kernels.
struct State {
    int32_t done, status, sweep_mode, vec_action;
    int32_t exp64, ls_phase, stage, reset;
    int32_t save_best, inner_warn, ls_trials_cur, standalone;  // standalone: 0 solve, 1 LSE only, 2 round+certify
    int32_t budget_stop, exp64_stage;
    int32_t on_proxy, sk_half;  // on_proxy: the stage runs on the FP16 copy of the cost (MIXED);
                                // sk_half: Sinkhorn projector, 1 after the row update of an iteration
    double gamma, gamma_prev, eps_d, w, ws_ratio, ws_scale, tol;
    double alpha, alpha_acc, alpha_prev, beta;
    double dphi0, alo, dlo, ahi, dhi, gnorm;
    double r1[4];   // R1 sums: c.g'(2), r.f''(2)
    double errc_sum;
    double best_ub, best_lb, best_gamma, best_me, last_ub, last_lb;
    double f32_floor;   // FP64 exp for stages with tolerance below this (raised by the stall guard)
    double stall_best;  // smallest ||grad||_1 of the stage when it last halved, at iteration stall_k
    int64_t k, sweeps, pncg_iters, ls_trials, cg_resets, ls_failures, fallbacks, cert_sweeps;
    int64_t stall_k, prec_switches, proxy_stages, tilde_iters;
};

// Device buffers of one problem (all FP64 unless noted). (m + n)-vectors hold the m rows, then
// the n columns: entry k < m is row k, entry m + j is column j.
struct Work {
    int32_t m, n, nrt, nct;  // rows (sources, r), columns (targets, c), row tiles, column tiles
    int32_t cost_kind, dtype, d, fin_per;  // cost kind and dtype, point dimension, fin_per(m, n)
    int32_t fin_Lr, fin_lgLr, fin_nvbr;  // fin_lanes_r(m, n), log2 of it, fin_vblocks_r(m, n)
    int32_t fin_L, fin_lgL, fin_nvb, fin_nblk;  // fin_lanes_c(m, n), log2 of it, fin_vblocks(m, n), fin_grid(m, n)
    // launch variant from the tuning table (neither changes any arithmetic): occ2 = 1 runs the
    // sweep instance capped at 2 waves per SIMD (256 VGPRs) instead of 4 (128 VGPRs); FP32 sweeps
    // of more than stage_min_tiles tiles stage their second row batch in LDS
    int32_t occ2, stage_min_tiles;
    const void* cost;        // dense cost or coordinates X then Y
    double scale;            // C = scale * raw
    const double* r;         // original marginals
    const double* c;
    double* rt;        // [m+n] smoothed marginals r~, c~
    double* logt;      // [m+n] log r~, log c~
    double* z;         // [m+n] u, v
    double* zprev;     // [m+n] previous-stage solution
    double* zbest;     // [m+n] potentials of the best UB stage
    double* p;         // [m+n] search direction
    double* g;         // [m+n] gradient at z
    double* lz;        // [m+n] log r(P), log c(P) at z (or a prediction)
    double* lzt;       // [m+n] at the current trial
    double* xr;        // [m]  Round row factors x
    double* yc;        // [n]  Round column factors y
    double* errc;      // [n]  err_c
    double* gp;        // [2n] g' (two variants, n apart) from R1
    double* fpp;       // [2m] f'' (two variants, m apart) from R1
    double* rowpart;   // [nct * m]    per-tile row partials (column tile J, row i at J m + i)
    double* colpart;   // [nrt * n]    per-tile column partials (row tile I, column j at I n + j)
    double* rowpart2;  // [nct * m]    second row partial (R2)
    double* rowpart3;  // [nct * m]    third row partial (R2)
    double* rowmin;    // [2 * nct * m] per-tile row minima (two variants)
    double* colmin;    // [2 * nrt * n] per-tile column minima
    double* tshift;    // [nrt] per-row-tile column shift S_I
    double* sdt;       // [m+n] diagonal-Hessian direction s~ at the current trial (precond variant)
    double* bdots;     // [fin_grid(m, n) * kNDot] per-workgroup dot products (in the control block)
    State* st;         // [2] state slots: step k reads slot k % 2, its decide kernel writes the other
    DevParams* prm;
};

// Control block of one problem in device memory: the Work struct followed, at fixed offsets,
// by the two state slots, the parameters and the finalize kernel's per-workgroup dots. Kernels
// address these from the Work pointer itself, so their loads need not wait for the Work load.
// Work::st, Work::prm and Work::bdots point at the same members.
struct Control {
    Work w;
    State st[2];
    DevParams prm;
    double bdots[kFinMaxGrid * kNDot];
};

// Problems in flight in one batched launch. Every item has its own Work, state slots and
// counters, so its results do not depend on the rest of the batch.
// Finalize: workgroup g belongs to item b with fin_prefix[b] <= g < fin_prefix[b+1].
// Sweep: the items are grouped by cost (same cost data, n and kind), and group q owns
// workgroups grp_prefix[q] <= g < grp_prefix[q+1] (grp_prefix is a multiple of 8). Within a
// group of K items with T tiles each, workgroup l = g - grp_prefix[q] sweeps tile
// t = 8 (l / 8 / K) + l % 8 of the group's item (l / 8) % K (idle when t >= T): the K sweeps of
// one cost tile land on the same XCD (workgroups go round-robin over the 8 XCDs) at nearly the
// same time, so the cost is read from HBM once per group and from that XCD's L2 by the rest.
constexpr int kMaxBatch = 64;
constexpr int kCostCodes = 10;           // cost types (dense dtypes; point metrics for d <= 3, d <= 2, d <= 8)
constexpr int kOccHi = 16;               // code bit: the same cost type at 2 waves per SIMD
constexpr int kMaxCodes = kOccHi + kCostCodes;  // sweep kernel instance codes (some unused)
constexpr int kStageMinTilesDefault = 2048;
struct BatchDesc {
    int32_t nitems, total_tiles, total_fin, ngroups;
    int32_t fin_prefix[kMaxBatch + 1];
    int32_t grp_prefix[kMaxBatch + 1];
    int32_t grp_first[kMaxBatch];  // first entry of the group in grp_items
    int32_t grp_size[kMaxBatch];   // K
    int32_t grp_tiles[kMaxBatch];  // T
    int32_t grp_items[kMaxBatch];  // item indices, group by group
    const Work* items[kMaxBatch];
    // Groups are ordered by the sweep kernel instance they need (cost code, planar when d <= 2):
    // instance code[c] sweeps the tiles [code_begin[c], code_begin[c + 1]).
    int32_t ncodes;
    int32_t code[kMaxCodes];
    int32_t code_begin[kMaxCodes + 1];
};

// Workspace layout of one problem (the vectors of Work, in the order bind_work assigns them):
// FP64 counts per buffer for m rows and n columns, each buffer rounded up to 256 bytes.
constexpr int kWsBuffers = 22;
constexpr size_t ws_count(int b, size_t m, size_t n)
{
    const size_t nrt = (m + kBR - 1) / kBR, nct = (n + kBC - 1) / kBC;
    return b < 9 ? m + n                      // rt logt z zprev zbest p g lz lzt
         : b == 9 ? m                         // xr
         : b < 12 ? n                         // yc errc
         : b == 12 ? 2 * n                    // gp
         : b == 13 ? 2 * m                    // fpp
         : b == 14 || b == 16 || b == 17 ? nct * m  // rowpart rowpart2 rowpart3
         : b == 15 ? nrt * n                  // colpart
         : b == 18 ? 2 * nct * m              // rowmin
         : b == 19 ? 2 * nrt * n              // colmin
         : b == 20 ? nrt                      // tshift
         : m + n;                             // sdt
}
constexpr size_t ws_round(size_t bytes) { return (bytes + 255) / 256 * 256; }
// Byte offset of buffer b (b = kWsBuffers gives the total).
constexpr size_t ws_offset(int b, size_t m, size_t n)
{
    size_t off = 0;
    for (int i = 0; i < b; ++i) off += ws_round(ws_count(i, m, n) * sizeof(double));
    return off;
}

// The allocation-free LSE entry point keeps its control block, workspace and cost-range
// partials in one static device array of kNoAllocBytes per device: the control block first,
// then the workspace of m = n = kNoAllocMaxN (which holds that of any m, n <= kNoAllocMaxN), then
// 2 partials per tile of that size.
constexpr int kNoAllocMaxN = MDOT_NOALLOC_MAX_N;
constexpr size_t kNoAllocCtl = ws_round(sizeof(Control));
constexpr size_t kNoAllocRange =
    ws_round(2 * sizeof(double) * ((kNoAllocMaxN + kBR - 1) / kBR) * ((kNoAllocMaxN + kBC - 1) / kBC));
constexpr size_t kNoAllocBytes = kNoAllocCtl + ws_offset(kWsBuffers, kNoAllocMaxN, kNoAllocMaxN) + kNoAllocRange;
// Device address of that array on the current device (hipGetSymbolAddress, taken once per
// device and cached). Returns 0 or a hipError_t code.
int noalloc_scratch(int device, void** out);
// Fill count doubles at dst with val (a kernel, so the fill is an ordinary kernel node if the
// caller's stream is being captured).
int launch_fill(double* dst, size_t count, double val, void* stream);
// Read count doubles at src (cache eviction for cold-cache timing); sink[0] is written only if
// their sum is -1.2345e300.
int launch_touch(const double* src, size_t count, double* sink, void* stream);

// Host-side launchers (mdot_kernels.hip). `hw` is the host copy of the Work struct (sizes
// and cost type pick the grid and the kernel instance), `wd` its device copy.
int launch_step(const Work& hw, const Work* wd, int parity, void* stream);  // sweep, finalize, decide
int launch_sweep(const Work& hw, const Work* wd, int parity, void* stream); // the LSE sweep kernel alone
int launch_init(const Work* wd, void* stream);                               // state + first stage
int launch_intake(const Work* wd, double* out8, void* stream);
int launch_cost_range(const Work& hw, const Work* wd, double* part, void* stream);
int launch_finish(const Work* wd, double* u_out, double* v_out, void* stream);
// FP16 copy of a dense FP32 (src_dtype MDOT_DT_F32) or FP64 cost; part[b] = max |C16 - C| of block b.
int launch_to_f16(const void* src, int src_dtype, void* dst, size_t count, double* part, int nblocks, void* stream);
// Batched step over a BatchDesc in device memory: one sweep launch per kernel instance of the
// host copy hb (instance hb.code[c] over its tile range), then fin_grid = total_fin finalize
// workgroups and the decisions.
int cost_code_of(int cost_kind, int dtype);
// The instance of a point cost code for dimension d (planar for d <= 2, the general one for
// d = 3, the 8-coordinate one for 4 <= d <= 8); other codes are returned unchanged.
int cost_code_dim(int cost_code, int d);
// The sweep kernel instance a launch of hw takes (its cost code, planar for d <= 2, plus kOccHi
// for the 2-waves-per-SIMD variant).
int cost_code(const Work& hw);
// fin_v: the finalize instance (fin_instance) the largest problem in flight needs
int launch_step_batch(const BatchDesc& hb, const BatchDesc* bd, int parity, int fin_grid, int fin_v, void* stream);
// End-of-chunk done flags into host-visible memory: chunk number *seq (a device counter, advanced
// here) writes out[(seq & 1) * kMaxBatch + item] (batch) or out[seq & 1] (single problem).
int launch_gather_done(const BatchDesc* bd, int* out, int* seq, void* stream);
int launch_chunk_done(const Work* wd, int* out, int* seq, void* stream);

}  // namespace mdot
