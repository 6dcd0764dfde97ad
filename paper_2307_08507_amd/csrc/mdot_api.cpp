// C ABI of libmdot (include/mdot.h): context, workspace, intake validation and the host
// side of the solve loop. All solver decisions are taken on the device (mdot_kernels.hip);
// the host replays a captured graph of solver steps and polls a done flag once per chunk,
// keeping two chunks in flight so the GPU never waits for the host.
//
// The serving engine (mdot_submit / mdot_run / mdot_poll) keeps up to kMaxBatch solves in
// flight. Every engine step advances all of them with one launch per kernel, one workgroup per
// tile and per finalize block of the solves in flight (a device batch descriptor maps
// workgroups to solves; the graph is captured again when the batch changes). A finished solve
// frees its slot when its chunk is read back, where new requests can be admitted if a slot and
// the HBM budget allow. Neither an admission nor a retirement waits for the chunk in flight:
// intake runs on a side stream, a retiring solve's potentials and state are copied out behind
// the chunk in flight (its workspace returns to the pool once that copy has completed), and
// the batch descriptor is uploaded from alternating host buffers.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mdot_internal.h"

using namespace mdot;

namespace {

constexpr int kChunk = 32;       // solver steps per graph launch (even: the state slot alternates)
constexpr int kBatchChunk = 16;  // engine steps per graph launch (admission granularity, even)
constexpr int kMaxN = MDOT_MAX_N;
constexpr int kConvBlocks = 1024; // workgroups of the FP16 conversion (MIXED)

// Device buffers of one problem: workspace, device copy of Work + 2 state slots, parameters.
struct ProblemBufs {
    bool borrowed = false;  // the buffers live in memory the context does not own (never freed)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int cap_n = 0;  // largest of m and n the workspace was bound for (pool ordering only)
    Work* d_work = nullptr;  // the Control block (Work, State[2], DevParams, dots)
    DevParams* d_prm = nullptr;  // inside the Control block
    Work host_work{};
    void* proxy = nullptr;  // MIXED: FP16 copy of the cost
    size_t proxy_bytes = 0;
};

// Device bytes a problem's buffers hold.
static size_t bufs_bytes(const ProblemBufs& pb)
{
    if (pb.borrowed) return 0;
    return (pb.d_work ? sizeof(Control) : 0) + pb.ws_bytes + pb.proxy_bytes;
}

// A solve whose chunk reported it finished: its finish kernel and the copy of its state into
// h_states[hs] are queued behind the chunk in flight, and `ev` is recorded after them. Its
// buffers return to the pool once `ev` has completed.
struct Retiring {
    ProblemBufs pb;
    uint64_t ticket = 0;
    int hs = 0;
};

struct Slot {
    bool used = false;
    uint64_t ticket = 0;
    ProblemBufs pb;
    double* u_out = nullptr;
    double* v_out = nullptr;
    size_t footprint = 0;
    // MIXED: the exact cost and the marginals, bound again when the solve pauses at the switch
    mdot_cost_desc exact{};
    const double* r = nullptr;
    const double* c = nullptr;
    int64_t resumed_at = -1;  // engine chunks up to this sequence number ran the paused state
};

}  // namespace

// One entry of the launch-variant table (written by paper_2307_08507_amd/tune.py): for cost
// type `code` (a base cost code, planar point codes separate) and sizes up to n_max, the sweep
// instance at 2 waves per SIMD (occ 2) or 4 (occ 4), and the LDS staging threshold in tiles.
struct TuneEntry {
    int code = 0, n_max = 0, occ = 4, stage_min_tiles = kStageMinTilesDefault;
};

struct mdot_ctx {
    int device = 0;
    std::vector<TuneEntry> tuning;  // sorted by (code, n_max)
    int force_occ = 0, force_stage = -1;  // mdot_tune_override
    hipStream_t stream = nullptr;
    size_t budget = 0;
    std::string err;
    ProblemBufs main;             // single solves and the standalone entry points
    // mdot_lse2_noalloc: its buffers are borrowed from the library's static device array, whose
    // address on this device was taken at context creation
    ProblemBufs fixed;
    unsigned char* d_fixed = nullptr;
    State* h_state = nullptr;     // pinned
    // done flags written by the last kernel of each graph chunk (pinned, mapped, fine-grained):
    // 2 for the single solves, then 2 x kMaxBatch for the engine; d_hdone is the device alias
    int* h_done = nullptr;
    int* d_hdone = nullptr;
    int* d_seq = nullptr;     // device chunk counters: [0] single solves, [1] engine
    uint64_t solo_seq = 0;    // host mirror of d_seq[0]
    double* h_scratch = nullptr;  // pinned, intake results
    double* d_scratch = nullptr;  // device, intake results / cost range partials
    size_t scratch_doubles = 0;
    DevParams* h_prm = nullptr;   // pinned
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipGraphExec_t graph = nullptr;  // captured chunk of solver steps for `main`
    // what the graph was captured with: m, n and the sweep kernel instance (cost code, which also
    // tells the point dimension classes apart)
    int graph_m = 0, graph_n = 0, graph_code = -1;
    // serving engine
    hipStream_t side = nullptr;     // intake of admitted solves (does not wait for the chunk in flight)
    Slot slots[kMaxBatch];
    std::vector<ProblemBufs> pool;  // released problem buffers kept for reuse
    std::vector<Retiring> retiring;
    State* h_states = nullptr;      // pinned, one state per retiring solve
    hipEvent_t ret_ev[kMaxBatch] = {};
    std::vector<int> free_hs;       // free indices of h_states / ret_ev
    BatchDesc* h_batch[2] = {nullptr, nullptr};  // pinned, alternating upload buffers
    hipEvent_t batch_ev[2] = {nullptr, nullptr};  // recorded after each buffer's upload
    int hb_cur = 0;                 // buffer holding the current descriptor
    BatchDesc* d_batch = nullptr;
    bool batch_dirty = true;
    hipGraphExec_t bgraph = nullptr;
    // replaced batch graphs, destroyed once the last chunk launched from them has been read back
    std::vector<std::pair<hipGraphExec_t, int64_t>> graveyard;
    // what the batch graph was captured with: its sweep instances and their tile ranges, the
    // finalize grid and finalize instance
    int bgraph_ncodes = 0, bgraph_code[kMaxCodes] = {}, bgraph_begin[kMaxCodes + 1] = {};
    int bgraph_fin = -1;
    int bgraph_fin_v = -1;
    int batch_fin_v = kFinSmall;  // the finalize instance the batch needs (fin_instance)
    // engine chunks in flight: the next chunk is launched before the previous one's done flags
    // are read; each remembers the slots and tickets it advanced, in descriptor order
    hipEvent_t eng_ev[2] = {nullptr, nullptr};
    int eng_pending = -1;  // buffer of the launched chunk not yet read back, or -1
    int eng_next = 0;      // buffer of the next chunk
    int64_t eng_seq = 0;              // engine chunks launched so far
    int64_t chunk_seq[2] = {0, 0};    // sequence number of the chunk in each buffer
    int chunk_m[2] = {0, 0};
    int chunk_slot[2][kMaxBatch];
    uint64_t chunk_ticket[2][kMaxBatch];
    uint64_t next_ticket = 1;
    size_t bytes_in_use = 0;  // buffers of the solves in slots and retiring
    std::map<uint64_t, mdot_result> finished;
};

static int fail(mdot_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIPCHK(ctx, call)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, MDOT_E_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                      \
    } while (0)

static inline int tiles_r(int n) { return (n + kBR - 1) / kBR; }
static inline int tiles_c(int n) { return (n + kBC - 1) / kBC; }

// Rows of a cost (m = 0 in the descriptor means square).
static inline int rows_of(const mdot_cost_desc* c) { return c->m > 0 ? c->m : c->n; }

// Bytes of workspace for m rows and n columns (see Work and ws_offset in mdot_internal.h);
// out_offsets, if given, receives the kWsBuffers + 1 buffer offsets.
static size_t workspace_bytes(int m, int n, size_t* out_offsets = nullptr)
{
    if (out_offsets)
        for (int i = 0; i <= kWsBuffers; ++i) out_offsets[i] = ws_offset(i, (size_t)m, (size_t)n);
    return ws_offset(kWsBuffers, (size_t)m, (size_t)n);
}

static size_t problem_footprint(int m, int n)
{
    return workspace_bytes(m, n) + sizeof(Control);
}

static void free_bufs(ProblemBufs& pb)
{
    if (pb.borrowed) {
        pb = ProblemBufs{};
        return;
    }
    if (pb.ws) (void)hipFree(pb.ws);
    if (pb.d_work) (void)hipFree(pb.d_work);
    if (pb.proxy) (void)hipFree(pb.proxy);
    pb = ProblemBufs{};
}

static int ensure_scratch(mdot_ctx* ctx, int m, int n)
{
    const size_t scr = std::max<size_t>(kConvBlocks, 2 * (size_t)tiles_r(m) * tiles_c(n));
    if (scr <= ctx->scratch_doubles) return MDOT_OK;
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    if (ctx->h_scratch) (void)hipHostFree(ctx->h_scratch);
    ctx->d_scratch = nullptr;
    ctx->h_scratch = nullptr;
    ctx->scratch_doubles = 0;
    HIPCHK(ctx, hipMalloc(&ctx->d_scratch, scr * sizeof(double)));
    HIPCHK(ctx, hipHostMalloc(&ctx->h_scratch, scr * sizeof(double), hipHostMallocDefault));
    ctx->scratch_doubles = scr;
    return MDOT_OK;
}

// Make pb hold a workspace for m rows and n columns (reallocating when it is too small).
static int ensure_workspace(mdot_ctx* ctx, ProblemBufs& pb, int m, int n, hipStream_t stream)
{
    if (!pb.d_work) {
        HIPCHK(ctx, hipMalloc(&pb.d_work, sizeof(Control)));
        pb.d_prm = &reinterpret_cast<Control*>(pb.d_work)->prm;
    }
    const size_t need = workspace_bytes(m, n);
    if (pb.ws && need <= pb.ws_bytes) return ensure_scratch(ctx, m, n);
    if (pb.ws) {
        (void)hipFree(pb.ws);
        pb.ws = nullptr;
        pb.ws_bytes = 0;
        pb.cap_n = 0;
    }
    if (ctx->graph) {  // the captured graph may reference the old sizes
        (void)hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
        ctx->graph_m = ctx->graph_n = 0;
    }
    hipError_t e = hipMalloc(&pb.ws, need);
    if (e != hipSuccess) {
        pb.ws = nullptr;
        return fail(ctx, MDOT_E_NOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
    }
    pb.ws_bytes = need;
    pb.cap_n = std::max(m, n);
    HIPCHK(ctx, hipMemsetAsync(pb.ws, 0, need, stream));
    return ensure_scratch(ctx, m, n);
}

// Names of the base cost codes in the tuning file (the order of CostCode in the kernels).
static const char* const kCodeNames[kCostCodes] = {"f64", "f32", "f16", "bf16", "pts_sq", "pts_l1", "pts_sq2",
                                                   "pts_l12", "pts_sq8", "pts_l18"};

// Read the tuning table: $MDOT_TUNING, else tuning.json in the package directory (the parent of
// the directory holding libmdot.so). The file is JSON written one entry per line by the tuner:
//   {"code": "f32", "n_max": 4096, "occ": 4, "stage_min_tiles": 2048, ...}
// Unknown fields are ignored; a missing or unreadable file leaves the built-in defaults (occ 4,
// staging above kStageMinTilesDefault tiles). The variants never change results.
static void load_tuning(mdot_ctx* ctx)
{
    std::string path;
    if (const char* env = std::getenv("MDOT_TUNING")) {
        path = env;
    } else {
        Dl_info info;
        if (dladdr((void*)&load_tuning, &info) && info.dli_fname) {
            std::string so = info.dli_fname;
            const size_t a = so.find_last_of('/');
            std::string dir = a == std::string::npos ? "." : so.substr(0, a);
            const size_t b = dir.find_last_of('/');
            path = (b == std::string::npos ? std::string(".") : dir.substr(0, b)) + "/tuning.json";
        }
    }
    FILE* f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    auto field = [](const char* l, const char* key, int* out) {
        const char* p = std::strstr(l, key);
        if (!p) return false;
        p = std::strchr(p + std::strlen(key), ':');
        return p && std::sscanf(p + 1, " %d", out) == 1;
    };
    while (std::fgets(line, sizeof line, f)) {
        const char* c = std::strstr(line, "\"code\"");
        if (!c) continue;
        char name[32] = {0};
        if (std::sscanf(std::strchr(c + 6, ':') + 1, " \"%31[^\"]\"", name) != 1) continue;
        TuneEntry e;
        e.code = -1;
        for (int k = 0; k < kCostCodes; ++k)
            if (!std::strcmp(name, kCodeNames[k])) e.code = k;
        if (e.code < 0 || !field(line, "\"n_max\"", &e.n_max) || !field(line, "\"occ\"", &e.occ) ||
            !field(line, "\"stage_min_tiles\"", &e.stage_min_tiles))
            continue;
        if (e.occ != 2 && e.occ != 4) continue;
        ctx->tuning.push_back(e);
    }
    std::fclose(f);
    std::sort(ctx->tuning.begin(), ctx->tuning.end(), [](const TuneEntry& a, const TuneEntry& b) {
        return a.code != b.code ? a.code < b.code : a.n_max < b.n_max;
    });
}

// The launch variant for base cost code `code` at size n: the first table entry of that code
// with n <= n_max (defaults if none), then the context's overrides.
static void pick_variant(const mdot_ctx* ctx, int code, int n, int* occ2, int* stage_min_tiles)
{
    // the 8-coordinate point instances hold 4 x 8 FP64 column coordinates per lane: they take the
    // 256-VGPR variant unless the table says otherwise
    int occ = (code == kCostCodes - 2 || code == kCostCodes - 1) ? 2 : 4, st = kStageMinTilesDefault;
    for (const TuneEntry& e : ctx->tuning)
        if (e.code == code && n <= e.n_max) {
            occ = e.occ;
            st = e.stage_min_tiles;
            break;
        }
    if (ctx->force_occ) occ = ctx->force_occ;
    if (ctx->force_stage == 0) st = 0x7fffffff;
    if (ctx->force_stage == 1) st = 0;
    *occ2 = occ == 2;
    *stage_min_tiles = st;
}

// Lay the Work struct out over pb's workspace for m rows and n columns (the workspace holds at
// least workspace_bytes(m, n)) and upload it.
static int bind_work(mdot_ctx* ctx, ProblemBufs& pb, int m, int n, const mdot_cost_desc* cost, double scale,
                     const double* r, const double* c, hipStream_t stream)
{
    size_t off[32];
    workspace_bytes(m, n, off);
    char* b = (char*)pb.ws;
    Work& w = pb.host_work;
    memset(&w, 0, sizeof w);
    w.m = m;
    w.n = n;
    w.nrt = tiles_r(m);
    w.nct = tiles_c(n);
    w.fin_Lr = fin_lanes_r(m, n);
    w.fin_L = fin_lanes_c(m, n);
    w.fin_per = fin_per(m, n);
    while ((1 << w.fin_lgLr) < w.fin_Lr) ++w.fin_lgLr;
    while ((1 << w.fin_lgL) < w.fin_L) ++w.fin_lgL;
    w.fin_nvbr = fin_vblocks_r(m, n);
    w.fin_nvb = fin_vblocks(m, n);
    w.fin_nblk = fin_grid(m, n);
    w.cost_kind = cost ? cost->kind : MDOT_COST_DENSE;
    w.dtype = cost ? cost->dtype : MDOT_DT_F32;
    w.d = cost ? cost->d : 0;
    {
        const int cc = cost_code_of(w.cost_kind, w.dtype);
        pick_variant(ctx, cost_code_dim(cc, w.d), std::max(m, n), &w.occ2, &w.stage_min_tiles);
    }
    w.cost = cost ? cost->data : nullptr;
    w.scale = scale;
    w.r = r;
    w.c = c;
    double** vec[] = {&w.rt, &w.logt, &w.z, &w.zprev, &w.zbest, &w.p, &w.g, &w.lz, &w.lzt, &w.xr, &w.yc,
                      &w.errc, &w.gp, &w.fpp, &w.rowpart, &w.colpart, &w.rowpart2, &w.rowpart3, &w.rowmin,
                      &w.colmin, &w.tshift, &w.sdt};
    const int k = sizeof(vec) / sizeof(vec[0]);
    static_assert(sizeof(vec) / sizeof(vec[0]) == kWsBuffers, "one workspace buffer per Work vector");
    for (int i = 0; i < k; ++i) *vec[i] = (double*)(b + off[i]);
    // standalone sweeps bind no marginals; point r and c at an n-vector of the workspace so
    // that no kernel can ever dereference a null pointer (their values are unused there)
    if (!w.r) w.r = w.xr;
    if (!w.c) w.c = w.yc;
    Control* ctl = reinterpret_cast<Control*>(pb.d_work);
    w.st = ctl->st;
    w.prm = &ctl->prm;
    w.bdots = ctl->bdots;
    HIPCHK(ctx, hipMemcpyAsync(pb.d_work, &w, sizeof w, hipMemcpyHostToDevice, stream));
    return MDOT_OK;
}

static void fill_defaults(mdot_params* p)
{
    p->p = 1.5;
    p->q = std::pow(2.0, 1.0 / 3.0);
    p->gamma_i = 16.0;
    p->gamma_f = 0.0;
    p->gamma_cap = 0.0;
    p->ls_c1 = 0.1;
    p->ls_c2 = 0.9;
    p->max_ls_trials = 50;
    p->max_pncg_iters = 100000;
    p->max_sweeps = 0;
    p->precision = MDOT_PREC_F32;
    p->warm_start = 1;
    p->mixed_switch = 0.05;
    p->projector = 0;
    p->precond = 0;
    p->smoothing = 0;
    p->tol_log_n = 0;
}

static int check_cost_desc(mdot_ctx* ctx, const mdot_cost_desc* cost)
{
    if (!cost || !cost->data) return fail(ctx, MDOT_E_ARG, "cost descriptor or its data is NULL");
    if (cost->n < 1 || cost->n > kMaxN) return fail(ctx, MDOT_E_ARG, "n=%d outside [1, %d]", cost->n, kMaxN);
    if (cost->m < 0 || cost->m > kMaxN) return fail(ctx, MDOT_E_ARG, "m=%d outside [0, %d]", cost->m, kMaxN);
    if (cost->reserved != 0) return fail(ctx, MDOT_E_ARG, "reserved field of the cost descriptor is not 0");
    if (cost->kind != MDOT_COST_DENSE && cost->kind != MDOT_COST_POINTS_SQEUCLID && cost->kind != MDOT_COST_POINTS_L1)
        return fail(ctx, MDOT_E_ARG, "unknown cost kind %d", (int)cost->kind);
    if (cost->kind == MDOT_COST_DENSE && (cost->dtype < MDOT_DT_F64 || cost->dtype > MDOT_DT_BF16))
        return fail(ctx, MDOT_E_ARG, "unknown dtype %d", (int)cost->dtype);
    if (cost->kind != MDOT_COST_DENSE && (cost->d < 1 || cost->d > 8))
        return fail(ctx, MDOT_E_ARG, "point dimension d=%d outside [1, 8]", cost->d);
    if (!(cost->scale >= 0.0) || !std::isfinite(cost->scale) || (cost->kind == MDOT_COST_DENSE && cost->scale == 0.0))
        return fail(ctx, MDOT_E_ARG, "bad cost scale %g", cost->scale);
    return MDOT_OK;
}

static int check_params(mdot_ctx* ctx, const mdot_params& prm, double target_gap)
{
    const bool adaptive = !(prm.gamma_f > 0.0);
    if (adaptive && !(target_gap > 0.0 && std::isfinite(target_gap)))
        return fail(ctx, MDOT_E_ARG, "target_gap must be > 0 in adaptive mode");
    if (!(prm.p >= 1.0) || !(prm.q > 1.0) || !(prm.gamma_i > 0.0) ||
        !(prm.ls_c1 > 0.0 && prm.ls_c1 < prm.ls_c2 && prm.ls_c2 < 1.0) || prm.max_ls_trials < 1 ||
        prm.max_pncg_iters < 1 || prm.max_sweeps < 0 ||
        (prm.precision != MDOT_PREC_F32 && prm.precision != MDOT_PREC_F64 && prm.precision != MDOT_PREC_MIXED) ||
        (prm.precision == MDOT_PREC_MIXED && !(prm.mixed_switch > 0.0 && std::isfinite(prm.mixed_switch))))
        return fail(ctx, MDOT_E_ARG, "invalid parameters");
    if (prm.warm_start < 0 || prm.warm_start > 2 || (prm.projector != 0 && prm.projector != 1) ||
        (prm.precond != 0 && prm.precond != 1) || (prm.smoothing != 0 && prm.smoothing != 1) ||
        (prm.tol_log_n != 0 && prm.tol_log_n != 1))
        return fail(ctx, MDOT_E_ARG, "invalid variant parameters (warm_start, projector, precond, smoothing, tol_log_n)");
    if (prm.projector == 1 && prm.precond == 1)
        return fail(ctx, MDOT_E_ARG, "precond applies to the PNCG projector only");
    return MDOT_OK;
}

// Range of the raw cost (one pass) -> resolved scale; MDOT_E_COST if scale*raw leaves [0,1].
// dpart: device buffer of 2 * tiles partials (the context's scratch unless given).
static int resolve_scale(mdot_ctx* ctx, ProblemBufs& pb, const mdot_cost_desc* cost, double* scale_out,
                         hipStream_t stream, double* dpart = nullptr)
{
    const int tiles = tiles_r(rows_of(cost)) * tiles_c(cost->n);
    if (!dpart) dpart = ctx->d_scratch;
    if (launch_cost_range(pb.host_work, pb.d_work, dpart, stream))
        return fail(ctx, MDOT_E_DEVICE, "cost range kernel launch failed");
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_scratch, dpart, 2 * tiles * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
    double lo = INFINITY, hi = -INFINITY;
    bool nonfinite = false;
    for (int t = 0; t < tiles; ++t) {
        lo = std::min(lo, ctx->h_scratch[2 * t]);
        const double h = ctx->h_scratch[2 * t + 1];
        if (std::isnan(h)) nonfinite = true;
        else hi = std::max(hi, h);
    }
    if (nonfinite || !std::isfinite(lo)) return fail(ctx, MDOT_E_COST, "cost has non-finite entries");
    double scale = cost->scale;
    if (cost->kind != MDOT_COST_DENSE && scale == 0.0) scale = hi > 0.0 ? 1.0 / hi : 1.0;
    const double slack = 1e-12;
    if (scale * lo < -slack || scale * hi > 1.0 + slack)
        return fail(ctx, MDOT_E_COST, "scaled cost range [%g, %g] is outside [0, 1]", scale * lo, scale * hi);
    *scale_out = scale;
    return MDOT_OK;
}

static int intake_marginals(mdot_ctx* ctx, ProblemBufs& pb, int m, int n, double* hmin, hipStream_t stream)
{
    if (launch_intake(pb.d_work, ctx->d_scratch, stream))
        return fail(ctx, MDOT_E_DEVICE, "intake kernel launch failed");
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_scratch, ctx->d_scratch, 8 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
    const double* s = ctx->h_scratch;
    const double tol = 1e-9 * std::max(m, n);
    if (s[6] > 0) return fail(ctx, MDOT_E_MARGINAL, "marginals contain non-finite values");
    if (s[2] < 0 || s[3] < 0) return fail(ctx, MDOT_E_MARGINAL, "marginals contain negative values");
    if (std::fabs(s[0] - 1.0) > tol || std::fabs(s[1] - 1.0) > tol)
        return fail(ctx, MDOT_E_MARGINAL, "marginals must sum to 1 (sum r = %.17g, sum c = %.17g)", s[0], s[1]);
    *hmin = std::min(s[4], s[5]);
    return MDOT_OK;
}

// Intake of one problem into pb on `stream`: workspace, Work, cost scale, marginal checks,
// parameters, initial state. Leaves the problem ready for its first solver step (state slot 0)
// and the stream idle.
static int setup_problem(mdot_ctx* ctx, ProblemBufs& pb, const mdot_cost_desc* cost, const double* r,
                         const double* c, double target_gap, const mdot_params& prm, hipStream_t stream)
{
    const int m = rows_of(cost), n = cost->n;
    int rc = ensure_workspace(ctx, pb, m, n, stream);
    if (rc) return rc;
    rc = bind_work(ctx, pb, m, n, cost, cost->scale > 0 ? cost->scale : 1.0, r, c, stream);
    if (rc) return rc;
    double scale;
    rc = resolve_scale(ctx, pb, cost, &scale, stream);
    if (rc) return rc;
    if (scale != pb.host_work.scale) {
        rc = bind_work(ctx, pb, m, n, cost, scale, r, c, stream);
        if (rc) return rc;
    }
    double hmin;
    rc = intake_marginals(ctx, pb, m, n, &hmin, stream);
    if (rc) return rc;
    const bool adaptive = !(prm.gamma_f > 0.0);
    DevParams& P = *ctx->h_prm;
    memset(&P, 0, sizeof P);
    P.p = prm.p;
    P.q = prm.q;
    P.gamma_i = prm.gamma_i;
    P.adaptive = adaptive;
    P.target = adaptive ? target_gap : 0.0;
    P.gamma_f = adaptive ? (prm.gamma_cap > 0.0 ? prm.gamma_cap : 5.0 * hmin / (2.0 * target_gap)) : prm.gamma_f;
    if (!(P.gamma_f > 0.0)) P.gamma_f = prm.gamma_i;  // H_min = 0: a single stage at gamma_i
    P.c1 = prm.ls_c1;
    P.c2 = prm.ls_c2;
    P.hmin = hmin;
    // App. C variant: log n in eps_d (log min(m, n), the upper bound of H_min, when m != n)
    P.hterm = prm.tol_log_n ? std::log((double)std::min(m, n)) : hmin;
    P.smooth_fixed = prm.smoothing == 1;
    P.w_fixed = std::min(P.hterm / std::pow(P.gamma_f, prm.p) / 4.0, 0.5);  // App. D: the final stage's weight
    P.projector = prm.projector;
    P.precond = prm.precond;
    P.tol_floor = 1e-14;
    P.f32_min_tol = 1e-7;  // about the L1 gradient resolution of FP32 exp sums
    P.max_sweeps = prm.max_sweeps;
    P.max_ls_trials = prm.max_ls_trials;
    P.max_pncg_iters = prm.max_pncg_iters;
    P.exp64_default = prm.precision == MDOT_PREC_F64;
    P.warm_start = prm.warm_start;
    P.n = n;
    if (prm.precision == MDOT_PREC_MIXED) {
        // FP16 copy of the cost and its largest rounding error delta; stages with
        // gamma * scale * delta <= mixed_switch run on the copy, and at least the last stage
        // before gamma_f runs on the exact cost
        const size_t count = (size_t)m * n;
        if (pb.proxy_bytes < count * 2) {
            if (pb.proxy) (void)hipFree(pb.proxy);
            pb.proxy = nullptr;
            pb.proxy_bytes = 0;
            HIPCHK(ctx, hipMalloc(&pb.proxy, count * 2));
            pb.proxy_bytes = count * 2;
        }
        if (launch_to_f16(cost->data, cost->dtype, pb.proxy, count, ctx->d_scratch, kConvBlocks, stream))
            return fail(ctx, MDOT_E_DEVICE, "conversion launch failed");
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_scratch, ctx->d_scratch, kConvBlocks * sizeof(double), hipMemcpyDeviceToHost,
                                   stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        double delta = 0.0;
        for (int b = 0; b < kConvBlocks; ++b) delta = std::max(delta, ctx->h_scratch[b]);
        const double scale = pb.host_work.scale;
        double mg = delta > 0.0 ? prm.mixed_switch / (scale * delta) : P.gamma_f;
        mg = std::min(mg, P.gamma_f / prm.q);
        P.mix_gamma = (mg >= std::min(P.gamma_i, P.gamma_f)) ? mg : 0.0;
    }
    HIPCHK(ctx, hipMemcpyAsync(pb.d_prm, &P, sizeof P, hipMemcpyHostToDevice, stream));
    if (launch_init(pb.d_work, stream)) return fail(ctx, MDOT_E_DEVICE, "init launch failed");
    if (P.mix_gamma > 0.0) {  // the first stages read the FP16 copy
        mdot_cost_desc proxy = *cost;
        proxy.dtype = MDOT_DT_F16;
        proxy.data = pb.proxy;
        const double scale = pb.host_work.scale;
        rc = bind_work(ctx, pb, m, n, &proxy, scale, r, c, stream);
        if (rc) return rc;
    }
    // the pinned parameter block is reused by the next intake: let this copy land first
    HIPCHK(ctx, hipStreamSynchronize(stream));
    return MDOT_OK;
}

static void fill_result(const State& S, double seconds, mdot_result* res)
{
    memset(res, 0, sizeof *res);
    res->primal_cost = S.best_ub;
    res->dual_bound = S.best_lb;
    res->gap = S.best_ub - S.best_lb;
    res->gamma_final = S.best_gamma;
    res->marg_err_l1 = S.best_me;
    res->grad_norm = S.gnorm;
    res->seconds = seconds;
    res->stages = S.stage;
    res->status = S.status;
    res->pncg_iters = S.pncg_iters;
    res->ls_trials = S.ls_trials;
    res->sweeps = S.sweeps;
    res->cg_resets = S.cg_resets;
    res->ls_failures = S.ls_failures;
    res->fp64_retries = S.fallbacks;
    res->cert_sweeps = S.cert_sweeps;
    res->prec_switches = S.prec_switches;
    res->proxy_stages = S.proxy_stages;
    res->tilde_iters = S.tilde_iters;
}

static int ensure_graph(mdot_ctx* ctx)
{
    const Work& hw = ctx->main.host_work;
    const int code = cost_code(hw);
    if (ctx->graph && ctx->graph_m == hw.m && ctx->graph_n == hw.n && ctx->graph_code == code) return MDOT_OK;
    if (ctx->graph) {
        (void)hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    hipStream_t cap;
    HIPCHK(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < kChunk; ++k) launch_step(hw, ctx->main.d_work, k & 1, cap);
        launch_chunk_done(ctx->main.d_work, ctx->d_hdone, ctx->d_seq, cap);
        e = hipStreamEndCapture(cap, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        ctx->graph = nullptr;
        return fail(ctx, MDOT_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    ctx->graph_m = hw.m;
    ctx->graph_n = hw.n;
    ctx->graph_code = code;
    return MDOT_OK;
}

// Run solver steps of `main` until the device sets done (or max_chunks chunks have run).
static int run_steps(mdot_ctx* ctx, int max_chunks)
{
    int rc = ensure_graph(ctx);
    if (rc) return rc;
    // slot 0 holds the newest state after an even chunk; the graph's last kernel copies its
    // done flag to h_done[chunk number & 1]
    const uint64_t base = ctx->solo_seq;
    int launched = 0, checked = 0;
    for (;;) {
        while (launched < checked + 2 && launched < max_chunks) {
            HIPCHK(ctx, hipGraphLaunch(ctx->graph, ctx->stream));
            HIPCHK(ctx, hipEventRecord(ctx->ev[launched & 1], ctx->stream));
            ++launched;
            ++ctx->solo_seq;
        }
        if (checked == launched) break;
        HIPCHK(ctx, hipEventSynchronize(ctx->ev[checked & 1]));
        const int done = ctx->h_done[(base + checked) & 1];
        ++checked;
        if (done) break;
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDOT_OK;
}

static int read_state(mdot_ctx* ctx, const ProblemBufs& pb)
{
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_state, pb.host_work.st, sizeof(State), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return MDOT_OK;
}

// ---------------------------------------------------------------- serving engine helpers
static int rebuild_batch(mdot_ctx* ctx)
{
    // the other host buffer: its last upload was queued at least one rebuild ago, behind a chunk
    // that has been read back since, so waiting for it does not wait for the chunk in flight
    const int hbuf = ctx->hb_cur ^ 1;
    HIPCHK(ctx, hipEventSynchronize(ctx->batch_ev[hbuf]));
    BatchDesc& B = *ctx->h_batch[hbuf];
    memset(&B, 0, sizeof B);
    int nf = 0, m = 0;
    const Work* hw[kMaxBatch];
    for (int s = 0; s < kMaxBatch; ++s) {  // items in slot order (the done flags follow it)
        const Slot& sl = ctx->slots[s];
        if (!sl.used) continue;
        hw[m] = &sl.pb.host_work;
        B.items[m] = sl.pb.d_work;
        B.fin_prefix[m] = nf;
        nf += sl.pb.host_work.fin_nblk;
        ++m;
    }
    B.nitems = m;
    B.fin_prefix[m] = nf;
    B.total_fin = nf;
    ctx->batch_fin_v = kFinSmall;
    for (int a = 0; a < m; ++a) ctx->batch_fin_v = std::max(ctx->batch_fin_v, fin_instance(hw[a]->fin_per, hw[a]->nrt));
    // sweep groups: items with the same cost data, size, point dimension, kind and dtype, in
    // order of first appearance; each needs one sweep kernel instance (planar for d <= 2 clouds)
    bool taken[kMaxBatch] = {};
    int gfirst[kMaxBatch], gcode[kMaxBatch], ngr = 0;
    for (int a = 0; a < m; ++a) {
        if (taken[a]) continue;
        for (int b = a; b < m; ++b) {
            const Work& x = *hw[a];
            const Work& y = *hw[b];
            if (y.cost == x.cost && y.m == x.m && y.n == x.n && y.d == x.d && y.cost_kind == x.cost_kind &&
                y.dtype == x.dtype)
                taken[b] = true;
        }
        const int code = cost_code(*hw[a]);  // includes the tuned occupancy variant
        if (code < 0 || code >= kMaxCodes)  // every code must get a tile range below
            return fail(ctx, MDOT_E_DEVICE, "cost code %d has no batched sweep range", code);
        gfirst[ngr] = a;
        gcode[ngr++] = code;
    }
    // lay the groups out instance by instance (one sweep launch per instance present)
    int ng = 0, ne = 0, nt = 0;
    B.ncodes = 0;
    for (int code = 0; code < kMaxCodes; ++code) {
        bool any = false;
        for (int q = 0; q < ngr; ++q) {
            if (gcode[q] != code) continue;
            if (!any) {
                B.code[B.ncodes] = code;
                B.code_begin[B.ncodes++] = nt;
                any = true;
            }
            const Work& x = *hw[gfirst[q]];
            B.grp_first[ng] = ne;
            B.grp_prefix[ng] = nt;
            int K = 0;
            for (int b = gfirst[q]; b < m; ++b) {
                const Work& y = *hw[b];
                if (y.cost != x.cost || y.m != x.m || y.n != x.n || y.d != x.d || y.cost_kind != x.cost_kind ||
                    y.dtype != x.dtype)
                    continue;
                B.grp_items[ne++] = b;
                ++K;
            }
            const int T = x.nrt * x.nct;
            B.grp_size[ng] = K;
            B.grp_tiles[ng] = T;
            nt += K * ((T + 7) / 8) * 8;
            ++ng;
        }
    }
    B.code_begin[B.ncodes] = nt;
    B.ngroups = ng;
    B.grp_prefix[ng] = nt;
    B.total_tiles = nt;
    // stream order puts the upload behind the chunk in flight, which still reads the old one
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_batch, &B, sizeof B, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->batch_ev[hbuf], ctx->stream));
    ctx->hb_cur = hbuf;
    ctx->batch_dirty = false;
    return MDOT_OK;
}

// The batch graph launches exactly one workgroup per tile and per finalize block of the
// problems in flight, one sweep launch per kernel instance, so it is captured again whenever
// the instances, their tile ranges or the totals change (admissions and completions, between
// chunks).
static int ensure_batch_graph(mdot_ctx* ctx)
{
    const BatchDesc& hb = *ctx->h_batch[ctx->hb_cur];
    const int fin = std::max(1, hb.total_fin);
    const int fin_v = ctx->batch_fin_v;
    bool same = ctx->bgraph && ctx->bgraph_ncodes == hb.ncodes && ctx->bgraph_fin == fin && ctx->bgraph_fin_v == fin_v;
    for (int c = 0; same && c < hb.ncodes; ++c)
        same = ctx->bgraph_code[c] == hb.code[c] && ctx->bgraph_begin[c + 1] == hb.code_begin[c + 1];
    if (same) return MDOT_OK;
    if (ctx->bgraph) {  // a chunk launched from it may still run: destroy it once that is read back
        ctx->graveyard.emplace_back(ctx->bgraph, ctx->eng_seq);
        ctx->bgraph = nullptr;
    }
    hipStream_t cap;
    HIPCHK(ctx, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < kBatchChunk; ++k) launch_step_batch(hb, ctx->d_batch, k & 1, fin, fin_v, cap);
        launch_gather_done(ctx->d_batch, ctx->d_hdone + 2, ctx->d_seq + 1, cap);
        e = hipStreamEndCapture(cap, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ctx->bgraph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        ctx->bgraph = nullptr;
        return fail(ctx, MDOT_E_DEVICE, "batch graph capture failed: %s", hipGetErrorString(e));
    }
    ctx->bgraph_ncodes = hb.ncodes;
    for (int c = 0; c < hb.ncodes; ++c) {
        ctx->bgraph_code[c] = hb.code[c];
        ctx->bgraph_begin[c + 1] = hb.code_begin[c + 1];
    }
    ctx->bgraph_fin = fin;
    ctx->bgraph_fin_v = fin_v;
    return MDOT_OK;
}

// Destroy the replaced batch graphs whose last chunk has been read back (chunk `seq` and
// everything launched before it have completed).
static void bury_graphs(mdot_ctx* ctx, int64_t seq)
{
    for (size_t k = 0; k < ctx->graveyard.size();) {
        if (ctx->graveyard[k].second <= seq) {
            (void)hipGraphExecDestroy(ctx->graveyard[k].first);
            ctx->graveyard.erase(ctx->graveyard.begin() + k);
        } else {
            ++k;
        }
    }
}

static void pool_put(mdot_ctx* ctx, const ProblemBufs& pb)
{
    ctx->pool.push_back(pb);
    // keep the pool bounded: free the smallest buffers beyond kMaxBatch entries
    while (ctx->pool.size() > (size_t)kMaxBatch) {
        auto it = std::min_element(ctx->pool.begin(), ctx->pool.end(),
                                   [](const ProblemBufs& a, const ProblemBufs& b) { return a.ws_bytes < b.ws_bytes; });
        free_bufs(*it);
        ctx->pool.erase(it);
    }
}

static size_t pool_bytes(const mdot_ctx* ctx)
{
    size_t b = 0;
    for (const ProblemBufs& pb : ctx->pool) b += bufs_bytes(pb);
    return b;
}

// Results of retiring solves whose state copies have completed (all of them with wait): the
// result becomes pollable and the buffers return to the pool. Adds the number collected to
// *collected (may be NULL).
static int collect_retired(mdot_ctx* ctx, bool wait, int* collected)
{
    for (size_t k = 0; k < ctx->retiring.size();) {
        Retiring& rt = ctx->retiring[k];
        hipError_t e = wait ? hipEventSynchronize(ctx->ret_ev[rt.hs]) : hipEventQuery(ctx->ret_ev[rt.hs]);
        if (e == hipErrorNotReady) {
            ++k;
            continue;
        }
        if (e != hipSuccess) return fail(ctx, MDOT_E_DEVICE, "retirement event failed: %s", hipGetErrorString(e));
        mdot_result res;
        fill_result(ctx->h_states[rt.hs], 0.0, &res);
        ctx->finished[rt.ticket] = res;
        ctx->bytes_in_use -= bufs_bytes(rt.pb);
        pool_put(ctx, rt.pb);
        ctx->free_hs.push_back(rt.hs);
        ctx->retiring.erase(ctx->retiring.begin() + k);
        if (collected) ++*collected;
    }
    return MDOT_OK;
}

// Retire the solve in `sl` (its chunk reported it finished): queue its finish kernel and the
// copy of its state behind the work in flight, free the slot, keep the buffers until the copy
// has completed.
static int retire_slot(mdot_ctx* ctx, Slot& sl)
{
    if (ctx->free_hs.empty()) {  // every state buffer is taken: wait for the oldest retirement
        int rc = collect_retired(ctx, true, nullptr);
        if (rc) return rc;
    }
    const int hs = ctx->free_hs.back();
    ctx->free_hs.pop_back();
    if (launch_finish(sl.pb.d_work, sl.u_out, sl.v_out, ctx->stream))
        return fail(ctx, MDOT_E_DEVICE, "finish launch failed");
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_states + hs, sl.pb.host_work.st, sizeof(State), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->ret_ev[hs], ctx->stream));
    Retiring rt;
    rt.pb = sl.pb;
    rt.ticket = sl.ticket;
    rt.hs = hs;
    ctx->retiring.push_back(rt);
    sl = Slot{};
    ctx->batch_dirty = true;
    return MDOT_OK;
}

extern "C" {

const char* mdot_version(void) { return "mdot-mi355x 0.2 (gfx950)"; }

void mdot_default_params(mdot_params* out)
{
    if (out) fill_defaults(out);
}

const char* mdot_last_error(const mdot_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mdot_tune_override(mdot_ctx* ctx, int occ, int stage)
{
    if (!ctx) return MDOT_E_ARG;
    if ((occ != 0 && occ != 2 && occ != 4) || stage < -1 || stage > 1)
        return fail(ctx, MDOT_E_ARG, "bad variant override (occ %d, stage %d)", occ, stage);
    ctx->force_occ = occ;
    ctx->force_stage = stage;
    return MDOT_OK;
}

int mdot_tune_variant(mdot_ctx* ctx, const mdot_cost_desc* cost, int* occ, int* stage_min_tiles)
{
    if (!ctx || !occ || !stage_min_tiles) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    const int cc = cost_code_of(cost->kind, cost->dtype);
    int o2 = 0;
    pick_variant(ctx, cost->kind != MDOT_COST_DENSE ? cost_code_dim(cc, cost->d) : cc, std::max(rows_of(cost), cost->n), &o2,
                 stage_min_tiles);
    *occ = o2 ? 2 : 4;
    return MDOT_OK;
}

int mdot_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, mdot_ctx** out)
{
    if (!out) return MDOT_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MDOT_E_DEVICE;
    if (device < 0 || device >= ndev) return MDOT_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return MDOT_E_DEVICE;
    mdot_ctx* ctx = new mdot_ctx();
    ctx->device = device;
    load_tuning(ctx);
    ctx->stream = (hipStream_t)hip_stream;
    ctx->budget = hbm_budget_bytes;
    bool ok = hipHostMalloc(&ctx->h_state, sizeof(State), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&ctx->h_prm, sizeof(DevParams), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&ctx->h_done, (2 * kMaxBatch + 2) * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) ==
                  hipSuccess &&
              hipHostGetDevicePointer((void**)&ctx->d_hdone, ctx->h_done, 0) == hipSuccess &&
              hipMalloc(&ctx->d_seq, 2 * sizeof(int)) == hipSuccess && hipMemset(ctx->d_seq, 0, 2 * sizeof(int)) == hipSuccess &&
              hipHostMalloc(&ctx->h_batch[0], sizeof(BatchDesc), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&ctx->h_batch[1], sizeof(BatchDesc), hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&ctx->h_states, kMaxBatch * sizeof(State), hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&ctx->d_batch, sizeof(BatchDesc)) == hipSuccess &&
              hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->batch_ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->batch_ev[1], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->ev[1], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->eng_ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->eng_ev[1], hipEventDisableTiming) == hipSuccess &&
              hipEventCreate(&ctx->t0) == hipSuccess && hipEventCreate(&ctx->t1) == hipSuccess;
    for (int k = 0; ok && k < kMaxBatch; ++k) {
        ok = hipEventCreateWithFlags(&ctx->ret_ev[k], hipEventDisableTiming) == hipSuccess;
        ctx->free_hs.push_back(kMaxBatch - 1 - k);
    }
    // address of the static array of mdot_lse2_noalloc on this device (taken once per device),
    // and the host and device scratch its cost-range pass uses, so that call allocates nothing
    void* fixed = nullptr;
    if (ok) ok = noalloc_scratch(device, &fixed) == 0 && fixed != nullptr;
    if (ok) ctx->d_fixed = static_cast<unsigned char*>(fixed);
    if (ok) ok = ensure_scratch(ctx, kNoAllocMaxN, kNoAllocMaxN) == MDOT_OK;
    if (!ok) {
        mdot_ctx_destroy(ctx);
        return MDOT_E_DEVICE;
    }
    *out = ctx;
    return MDOT_OK;
}

int mdot_ctx_destroy(mdot_ctx* ctx)
{
    if (!ctx) return MDOT_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
    if (ctx->bgraph) (void)hipGraphExecDestroy(ctx->bgraph);
    for (auto& g : ctx->graveyard) (void)hipGraphExecDestroy(g.first);
    free_bufs(ctx->main);
    for (auto& sl : ctx->slots)
        if (sl.used) free_bufs(sl.pb);
    for (auto& rt : ctx->retiring) free_bufs(rt.pb);
    for (auto& pb : ctx->pool) free_bufs(pb);
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    if (ctx->h_scratch) (void)hipHostFree(ctx->h_scratch);
    if (ctx->h_state) (void)hipHostFree(ctx->h_state);
    if (ctx->h_prm) (void)hipHostFree(ctx->h_prm);
    if (ctx->h_done) (void)hipHostFree(ctx->h_done);
    for (auto& hb : ctx->h_batch)
        if (hb) (void)hipHostFree(hb);
    if (ctx->h_states) (void)hipHostFree(ctx->h_states);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    for (auto& e : ctx->batch_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->ret_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->d_batch) (void)hipFree(ctx->d_batch);
    if (ctx->d_seq) (void)hipFree(ctx->d_seq);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : ctx->eng_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->t0) (void)hipEventDestroy(ctx->t0);
    if (ctx->t1) (void)hipEventDestroy(ctx->t1);
    delete ctx;
    return MDOT_OK;
}

int mdot_solve(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* r, const double* c, double target_gap,
               const mdot_params* params, double* u_out, double* v_out, mdot_result* res)
{
    if (!ctx) return MDOT_E_ARG;
    if (!res) return fail(ctx, MDOT_E_ARG, "result pointer is NULL");
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (!r || !c) return fail(ctx, MDOT_E_ARG, "marginal pointer is NULL");
    mdot_params prm;
    if (params) prm = *params;
    else fill_defaults(&prm);
    rc = check_params(ctx, prm, target_gap);
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int m = rows_of(cost), n = cost->n;
    // the single-problem buffers plus MIXED's FP16 copy, beside what the serving engine holds
    const size_t need = problem_footprint(m, n) + (prm.precision == MDOT_PREC_MIXED ? (size_t)m * n * 2 : 0);
    if (ctx->budget && need + ctx->bytes_in_use > ctx->budget) {
        for (auto& pb : ctx->pool) free_bufs(pb);  // idle engine buffers go first
        ctx->pool.clear();
    }
    if (ctx->budget && need + ctx->bytes_in_use > ctx->budget)
        return fail(ctx, MDOT_E_NOMEM, "m=%d n=%d needs %zu bytes, budget %zu has %zu in use", m, n, need,
                    ctx->budget, ctx->bytes_in_use);
    if (prm.precision == MDOT_PREC_MIXED &&
        (cost->kind != MDOT_COST_DENSE || (cost->dtype != MDOT_DT_F32 && cost->dtype != MDOT_DT_F64)))
        return fail(ctx, MDOT_E_ARG, "MIXED needs a dense FP32 or FP64 cost");
    rc = setup_problem(ctx, ctx->main, cost, r, c, target_gap, prm, ctx->stream);
    if (rc) return rc;
    HIPCHK(ctx, hipEventRecord(ctx->t0, ctx->stream));
    // hard cap on steps: every LSE sweep is one step, each stage adds at most a few more
    const int64_t max_steps = prm.max_sweeps > 0 ? 4 * prm.max_sweeps + 4096 : (int64_t)1 << 22;
    const int max_chunks = (int)std::min<int64_t>(max_steps / kChunk + 1, 1 << 30);
    rc = run_steps(ctx, max_chunks);
    if (rc) return rc;
    if (ctx->main.host_work.dtype != cost->dtype) {  // MIXED: paused at the switch to the exact cost
        rc = read_state(ctx, ctx->main);
        if (rc) return rc;
        if (ctx->h_state->done == 2) {
            rc = bind_work(ctx, ctx->main, m, n, cost, ctx->main.host_work.scale, r, c, ctx->stream);
            if (rc) return rc;
            static const int32_t kResume = 0;
            HIPCHK(ctx, hipMemcpyAsync(&ctx->main.host_work.st[0].done, &kResume, sizeof kResume,
                                       hipMemcpyHostToDevice, ctx->stream));
            rc = run_steps(ctx, max_chunks);
            if (rc) return rc;
        }
    }
    if (launch_finish(ctx->main.d_work, u_out, v_out, ctx->stream))
        return fail(ctx, MDOT_E_DEVICE, "finish launch failed");
    HIPCHK(ctx, hipEventRecord(ctx->t1, ctx->stream));
    rc = read_state(ctx, ctx->main);
    if (rc) return rc;
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    const State& S = *ctx->h_state;
    if (!S.done) return fail(ctx, MDOT_E_DEVICE, "solve did not finish within the step cap");
    fill_result(S, ms * 1e-3, res);
    return S.status;
}

// Set up pb for a standalone sweep sequence (one LSE, or Round + certificate). pb is the
// context's `main` (workspace allocated on demand) or its `fixed` buffers (borrowed from the
// static array: nothing is allocated, and the cost range partials go to `dpart` in that array).
static int standalone_setup(mdot_ctx* ctx, ProblemBufs& pb, const mdot_cost_desc* cost, const double* u,
                            const double* v, double gamma, const double* shift, int exp64, int kind,
                            const double* u_prev, const double* v_prev, double gamma_prev, const double* r,
                            const double* c, double* dpart = nullptr)
{
    const int m = rows_of(cost), n = cost->n;
    if (!pb.borrowed) {
        int rc = ensure_workspace(ctx, pb, m, n, ctx->stream);
        if (rc) return rc;
    }
    int rc = bind_work(ctx, pb, m, n, cost, cost->scale > 0 ? cost->scale : 1.0, r, c, ctx->stream);
    if (rc) return rc;
    double scale;
    rc = resolve_scale(ctx, pb, cost, &scale, ctx->stream, dpart);
    if (rc) return rc;
    if (scale != pb.host_work.scale) {
        rc = bind_work(ctx, pb, m, n, cost, scale, r, c, ctx->stream);
        if (rc) return rc;
    }
    const Work& w = pb.host_work;
    // rt .. lzt and the n-vectors xr, yc, errc (the vectors these sweeps read besides z and lz)
    // start at zero: a fill kernel, since the static array keeps the previous call's contents
    size_t off[kWsBuffers + 1];
    workspace_bytes(m, n, off);
    if (launch_fill(w.rt, off[12] / sizeof(double), 0.0, ctx->stream))
        return fail(ctx, MDOT_E_DEVICE, "fill launch failed");
    HIPCHK(ctx, hipMemcpyAsync(w.z, u, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(w.z + m, v, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    if (shift) HIPCHK(ctx, hipMemcpyAsync(w.lz, shift, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    const bool ext = u_prev && v_prev && gamma > gamma_prev;
    if (ext) {
        HIPCHK(ctx, hipMemcpyAsync(w.zprev, u_prev, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(w.zprev + m, v_prev, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    }
    DevParams& P = *ctx->h_prm;
    memset(&P, 0, sizeof P);
    P.exp64_default = exp64;
    P.n = n;
    P.gamma_f = gamma;
    HIPCHK(ctx, hipMemcpyAsync(pb.d_prm, &P, sizeof P, hipMemcpyHostToDevice, ctx->stream));
    State& S = *ctx->h_state;
    memset(&S, 0, sizeof S);
    S.standalone = kind;
    S.sweep_mode = shift ? SM_LSE : SM_MAX;
    S.ls_phase = LS_STANDALONE;
    S.exp64 = exp64;
    S.exp64_stage = exp64;
    S.gamma = gamma;
    S.gamma_prev = ext ? gamma_prev : gamma;
    S.best_ub = INFINITY;
    S.best_lb = -INFINITY;
    HIPCHK(ctx, hipMemcpyAsync(w.st, &S, sizeof S, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));  // the pinned blocks are reused later
    return MDOT_OK;
}

int mdot_lse2(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
              const double* shift, mdot_precision precision, double* lr_out, double* lc_out)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (!u || !v || !lr_out || !lc_out) return fail(ctx, MDOT_E_ARG, "NULL vector pointer");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(ctx, MDOT_E_ARG, "bad gamma %g", gamma);
    if (precision != MDOT_PREC_F32 && precision != MDOT_PREC_F64) return fail(ctx, MDOT_E_ARG, "bad precision");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    rc = standalone_setup(ctx, ctx->main, cost, u, v, gamma, shift, precision == MDOT_PREC_F64, 1, nullptr, nullptr, 0.0, nullptr,
                          nullptr);
    if (rc) return rc;
    rc = run_steps(ctx, 1);
    if (rc) return rc;
    rc = read_state(ctx, ctx->main);
    if (rc) return rc;
    if (!ctx->h_state->done) return fail(ctx, MDOT_E_DEVICE, "standalone sweep did not finish");
    const Work& w = ctx->main.host_work;
    const int m = rows_of(cost), n = cost->n;
    HIPCHK(ctx, hipMemcpyAsync(lr_out, w.lzt, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(lc_out, w.lzt + m, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return ctx->h_state->status;
}

int mdot_lse2_noalloc(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
                      const double* shift, mdot_precision precision, double* lr_out, double* lc_out)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (cost->n > kNoAllocMaxN || rows_of(cost) > kNoAllocMaxN)
        return fail(ctx, MDOT_E_ARG, "mdot_lse2_noalloc: m=%d n=%d exceeds its maximum %d (MDOT_NOALLOC_MAX_N)",
                    rows_of(cost), cost->n, kNoAllocMaxN);
    if (!u || !v || !lr_out || !lc_out) return fail(ctx, MDOT_E_ARG, "NULL vector pointer");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(ctx, MDOT_E_ARG, "bad gamma %g", gamma);
    if (precision != MDOT_PREC_F32 && precision != MDOT_PREC_F64) return fail(ctx, MDOT_E_ARG, "bad precision");
    if (!ctx->d_fixed) return fail(ctx, MDOT_E_DEVICE, "no static scratch on device %d", ctx->device);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    ProblemBufs& pb = ctx->fixed;
    pb.borrowed = true;
    pb.d_work = reinterpret_cast<Work*>(ctx->d_fixed);
    pb.d_prm = &reinterpret_cast<Control*>(ctx->d_fixed)->prm;
    pb.ws = ctx->d_fixed + kNoAllocCtl;
    pb.ws_bytes = workspace_bytes(rows_of(cost), cost->n);
    pb.cap_n = kNoAllocMaxN;
    double* dpart =
        reinterpret_cast<double*>(ctx->d_fixed + kNoAllocCtl + ws_offset(kWsBuffers, kNoAllocMaxN, kNoAllocMaxN));
    rc = standalone_setup(ctx, pb, cost, u, v, gamma, shift, precision == MDOT_PREC_F64, 1, nullptr, nullptr, 0.0,
                          nullptr, nullptr, dpart);
    if (rc) return rc;
    // at most three steps do work (row-max pass, LSE sweep, its FP64 re-run); later steps carry
    // the finished state over, and after an even number of steps slot 0 holds the newest state
    const Work& w = pb.host_work;
    for (int k = 0; k < 4; ++k)
        if (launch_step(w, pb.d_work, k & 1, ctx->stream)) return fail(ctx, MDOT_E_DEVICE, "step launch failed");
    rc = read_state(ctx, pb);
    if (rc) return rc;
    if (!ctx->h_state->done) return fail(ctx, MDOT_E_DEVICE, "standalone sweep did not finish");
    const int m = rows_of(cost), n = cost->n;
    HIPCHK(ctx, hipMemcpyAsync(lr_out, w.lzt, m * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(lc_out, w.lzt + m, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return ctx->h_state->status;
}

int mdot_round_certify(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
                       const double* u_prev, const double* v_prev, double gamma_prev, const double* r,
                       const double* c, double* ub, double* lb, double* marg_err)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (!u || !v || !r || !c || !ub || !lb || !marg_err) return fail(ctx, MDOT_E_ARG, "NULL pointer argument");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(ctx, MDOT_E_ARG, "bad gamma %g", gamma);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    rc = standalone_setup(ctx, ctx->main, cost, u, v, gamma, nullptr, 1, 2, u_prev, v_prev, gamma_prev, r, c);
    if (rc) return rc;
    rc = run_steps(ctx, 1);
    if (rc) return rc;
    rc = read_state(ctx, ctx->main);
    if (rc) return rc;
    if (!ctx->h_state->done) return fail(ctx, MDOT_E_DEVICE, "round/certify sweeps did not finish");
    *ub = ctx->h_state->best_ub;
    *lb = ctx->h_state->best_lb;
    *marg_err = ctx->h_state->best_me;
    return ctx->h_state->status;
}

int mdot_bench_sweep(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v, double gamma,
                     mdot_precision precision, int iters, double* ms_per_sweep)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (!u || !v || !ms_per_sweep || iters < 1) return fail(ctx, MDOT_E_ARG, "bad argument");
    if (precision != MDOT_PREC_F32 && precision != MDOT_PREC_F64) return fail(ctx, MDOT_E_ARG, "bad precision");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int exp64 = precision == MDOT_PREC_F64;
    // exact log-sums first (max pass + LSE pass) so the timed sweeps run with converged shifts
    rc = standalone_setup(ctx, ctx->main, cost, u, v, gamma, nullptr, exp64, 1, nullptr, nullptr, 0.0, nullptr, nullptr);
    if (rc) return rc;
    rc = run_steps(ctx, 1);
    if (rc) return rc;
    const Work& w = ctx->main.host_work;
    const int mn = rows_of(cost) + cost->n;
    HIPCHK(ctx, hipMemcpyAsync(w.lz, w.lzt, mn * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    State& S = *ctx->h_state;
    HIPCHK(ctx, hipMemcpyAsync(&S, w.st, sizeof S, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    S.done = 0;
    S.standalone = 1;
    S.sweep_mode = SM_LSE;
    S.ls_phase = LS_STANDALONE;
    S.exp64 = exp64;
    S.vec_action = 0;
    HIPCHK(ctx, hipMemcpyAsync(w.st, &S, sizeof S, hipMemcpyHostToDevice, ctx->stream));
    for (int k = 0; k < 3; ++k)
        if (launch_sweep(w, ctx->main.d_work, 0, ctx->stream)) return fail(ctx, MDOT_E_DEVICE, "sweep launch failed");
    HIPCHK(ctx, hipEventRecord(ctx->t0, ctx->stream));
    for (int k = 0; k < iters; ++k)
        if (launch_sweep(w, ctx->main.d_work, 0, ctx->stream)) return fail(ctx, MDOT_E_DEVICE, "sweep launch failed");
    HIPCHK(ctx, hipEventRecord(ctx->t1, ctx->stream));
    HIPCHK(ctx, hipEventSynchronize(ctx->t1));
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    *ms_per_sweep = (double)ms / iters;
    return MDOT_OK;
}

int mdot_bench_sweep_flushed(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* u, const double* v,
                             double gamma, mdot_precision precision, int iters, const void* flush, size_t flush_bytes,
                             double* ms_per_sweep)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    constexpr int kMaxIters = 256;
    if (!u || !v || !ms_per_sweep || iters < 1 || iters > kMaxIters || !flush || flush_bytes < sizeof(double))
        return fail(ctx, MDOT_E_ARG, "bad argument");
    if (precision != MDOT_PREC_F32 && precision != MDOT_PREC_F64) return fail(ctx, MDOT_E_ARG, "bad precision");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int exp64 = precision == MDOT_PREC_F64;
    rc = standalone_setup(ctx, ctx->main, cost, u, v, gamma, nullptr, exp64, 1, nullptr, nullptr, 0.0, nullptr, nullptr);
    if (rc) return rc;
    rc = run_steps(ctx, 1);
    if (rc) return rc;
    const Work& w = ctx->main.host_work;
    const int mn = rows_of(cost) + cost->n;
    HIPCHK(ctx, hipMemcpyAsync(w.lz, w.lzt, mn * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    State& S = *ctx->h_state;
    HIPCHK(ctx, hipMemcpyAsync(&S, w.st, sizeof S, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    S.done = 0;
    S.standalone = 1;
    S.sweep_mode = SM_LSE;
    S.ls_phase = LS_STANDALONE;
    S.exp64 = exp64;
    S.vec_action = 0;
    HIPCHK(ctx, hipMemcpyAsync(w.st, &S, sizeof S, hipMemcpyHostToDevice, ctx->stream));
    std::vector<hipEvent_t> ev(2 * iters, nullptr);
    int made = 0;
    for (; made < 2 * iters; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) break;
    auto cleanup = [&]() {
        for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
    };
    if (made < 2 * iters) {
        cleanup();
        return fail(ctx, MDOT_E_DEVICE, "event creation failed");
    }
    const size_t count = flush_bytes / sizeof(double);
    double* sink = reinterpret_cast<double*>(const_cast<void*>(flush));
    int lrc = 0;
    for (int k = 0; k < iters && !lrc; ++k) {
        // evict the cost from the L2s and the last-level cache by reading other data: the sweep
        // then streams it from HBM, with no dirty lines to write back
        lrc |= launch_touch(static_cast<const double*>(flush), count, sink, ctx->stream);
        lrc |= (int)hipEventRecord(ev[2 * k], ctx->stream);
        lrc |= launch_sweep(w, ctx->main.d_work, 0, ctx->stream);
        lrc |= (int)hipEventRecord(ev[2 * k + 1], ctx->stream);
    }
    if (lrc || hipStreamSynchronize(ctx->stream) != hipSuccess) {
        cleanup();
        return fail(ctx, MDOT_E_DEVICE, "flushed sweep timing failed");
    }
    double total = 0.0;
    for (int k = 0; k < iters; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) {
            cleanup();
            return fail(ctx, MDOT_E_DEVICE, "event timing failed");
        }
        total += ms;
    }
    cleanup();
    *ms_per_sweep = total / iters;
    return MDOT_OK;
}

// ---------------------------------------------------------------- serving engine
int mdot_submit(mdot_ctx* ctx, const mdot_cost_desc* cost, const double* r, const double* c, double target_gap,
                const mdot_params* params, double* u_out, double* v_out, uint64_t* ticket)
{
    if (!ctx) return MDOT_E_ARG;
    if (!ticket) return fail(ctx, MDOT_E_ARG, "ticket pointer is NULL");
    int rc = check_cost_desc(ctx, cost);
    if (rc) return rc;
    if (!r || !c) return fail(ctx, MDOT_E_ARG, "marginal pointer is NULL");
    mdot_params prm;
    if (params) prm = *params;
    else fill_defaults(&prm);
    rc = check_params(ctx, prm, target_gap);
    if (rc) return rc;
    if (prm.precision == MDOT_PREC_MIXED &&
        (cost->kind != MDOT_COST_DENSE || (cost->dtype != MDOT_DT_F32 && cost->dtype != MDOT_DT_F64)))
        return fail(ctx, MDOT_E_ARG, "MIXED needs a dense FP32 or FP64 cost");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int m = rows_of(cost), n = cost->n;
    const bool mixed = prm.precision == MDOT_PREC_MIXED;
    const size_t proxy_need = mixed ? (size_t)m * n * 2 : 0;  // MIXED also holds an FP16 copy of the cost
    const size_t ws_need = workspace_bytes(m, n);
    const size_t fp = problem_footprint(m, n) + proxy_need;
    if (ctx->budget && fp > ctx->budget)
        return fail(ctx, MDOT_E_NOMEM, "m=%d n=%d needs %zu bytes > budget %zu", m, n, fp, ctx->budget);
    rc = collect_retired(ctx, false, nullptr);  // finished retirements return their buffers first
    if (rc) return rc;
    int active = 0;
    for (const Slot& sl : ctx->slots) active += sl.used;
    if (active == kMaxBatch) return fail(ctx, MDOT_E_BUSY, "no free slot (%d solves in flight)", active);
    // reuse the smallest pooled workspace that fits. Every buffer the engine holds counts against
    // the budget at its actual size: solves in flight, retiring and pooled.
    auto pick = [&]() {
        int best = -1;
        for (int k = 0; k < (int)ctx->pool.size(); ++k)
            if (ctx->pool[k].ws_bytes >= ws_need && (best < 0 || ctx->pool[k].ws_bytes < ctx->pool[best].ws_bytes))
                best = k;
        return best;
    };
    auto held_after = [&](int cand) {
        const size_t held = ctx->bytes_in_use + pool_bytes(ctx);
        if (cand < 0) return held + fp;
        const ProblemBufs& pb = ctx->pool[cand];
        return held - bufs_bytes(pb) + sizeof(Control) + pb.ws_bytes + std::max(pb.proxy_bytes, proxy_need);
    };
    int best = pick();
    if (ctx->budget && held_after(best) > ctx->budget) {
        // the pool is idle memory: free it (all but the candidate, then the candidate too) before refusing
        for (int k = (int)ctx->pool.size() - 1; k >= 0; --k) {
            if (k == best) continue;
            free_bufs(ctx->pool[k]);
            ctx->pool.erase(ctx->pool.begin() + k);
            if (best > k) --best;
        }
        if (held_after(best) > ctx->budget && best >= 0) {
            free_bufs(ctx->pool[best]);
            ctx->pool.erase(ctx->pool.begin() + best);
            best = -1;
        }
        if (held_after(best) > ctx->budget)
            return fail(ctx, MDOT_E_BUSY, "HBM budget: %zu of %zu bytes in use, m=%d n=%d needs %zu",
                        ctx->bytes_in_use, ctx->budget, m, n, fp);
    }
    int s = 0;
    while (ctx->slots[s].used) ++s;
    Slot& sl = ctx->slots[s];
    if (best >= 0) {
        sl.pb = ctx->pool[best];
        ctx->pool.erase(ctx->pool.begin() + best);
    }
    // intake on the side stream: the buffers are idle (fresh, or pooled after their retirement
    // completed), so it need not wait for the chunk in flight on the context stream
    rc = setup_problem(ctx, sl.pb, cost, r, c, target_gap, prm, ctx->side);
    if (rc) {
        if (sl.pb.d_work) pool_put(ctx, sl.pb);
        sl = Slot{};
        return rc;
    }
    sl.used = true;
    sl.ticket = ctx->next_ticket++;
    sl.u_out = u_out;
    sl.v_out = v_out;
    sl.footprint = bufs_bytes(sl.pb);
    sl.exact = *cost;
    sl.r = r;
    sl.c = c;
    sl.resumed_at = -1;
    ctx->bytes_in_use += sl.footprint;
    ctx->batch_dirty = true;
    *ticket = sl.ticket;
    return MDOT_OK;
}

// Read back an engine chunk: retire the solves it finished (their slots may already hold newer
// solves, admitted after the chunk was launched: those are told apart by the ticket).
static int process_chunk(mdot_ctx* ctx, int buf)
{
    HIPCHK(ctx, hipEventSynchronize(ctx->eng_ev[buf]));
    bury_graphs(ctx, ctx->chunk_seq[buf]);
    const int* done = ctx->h_done + 2 + buf * kMaxBatch;
    for (int m = 0; m < ctx->chunk_m[buf]; ++m) {
        Slot& sl = ctx->slots[ctx->chunk_slot[buf][m]];
        if (!done[m] || !sl.used || sl.ticket != ctx->chunk_ticket[buf][m]) continue;
        if (done[m] == 2) {  // MIXED: paused at the switch to the exact cost
            // the chunk launched before the resume below still reports the pause: skip it
            if (ctx->chunk_seq[buf] <= sl.resumed_at) continue;
            int rc = bind_work(ctx, sl.pb, rows_of(&sl.exact), sl.exact.n, &sl.exact, sl.pb.host_work.scale, sl.r, sl.c,
                               ctx->stream);
            if (rc) return rc;
            // chunks have an even number of steps, so the next step reads state slot 0
            static const int32_t kResume = 0;
            HIPCHK(ctx, hipMemcpyAsync(&sl.pb.host_work.st[0].done, &kResume, sizeof kResume, hipMemcpyHostToDevice,
                                       ctx->stream));
            sl.resumed_at = ctx->eng_seq;
            ctx->batch_dirty = true;  // its sweep group now needs the exact cost's kernel instance
            continue;
        }
        int rc = retire_slot(ctx, sl);
        if (rc) return rc;
    }
    return MDOT_OK;
}

int mdot_run(mdot_ctx* ctx, int steps, int* n_done)
{
    if (!ctx) return MDOT_E_ARG;
    if (n_done) *n_done = 0;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    int completed = 0;
    int rc = collect_retired(ctx, false, &completed);
    if (rc) return rc;
    const int chunks = std::max(1, (steps + kBatchChunk - 1) / kBatchChunk);
    for (int ch = 0; ch < chunks; ++ch) {
        int active = 0;
        for (const Slot& sl : ctx->slots) active += sl.used;
        if (active == 0 && ctx->eng_pending < 0) break;
        if (active > 0) {  // launch the next chunk before reading the previous one back
            if (ctx->batch_dirty) {
                rc = rebuild_batch(ctx);
                if (rc) return rc;
            }
            rc = ensure_batch_graph(ctx);
            if (rc) return rc;
            const int buf = ctx->eng_next;
            int m = 0;
            for (int s = 0; s < kMaxBatch; ++s) {  // descriptor order = slot order
                if (!ctx->slots[s].used) continue;
                ctx->chunk_slot[buf][m] = s;
                ctx->chunk_ticket[buf][m] = ctx->slots[s].ticket;
                ++m;
            }
            ctx->chunk_m[buf] = m;
            ctx->chunk_seq[buf] = ++ctx->eng_seq;
            // the graph's last kernel writes this chunk's done flags to host buffer `buf` (engine
            // chunks alternate buffers in launch order, as the device counter does)
            HIPCHK(ctx, hipGraphLaunch(ctx->bgraph, ctx->stream));
            HIPCHK(ctx, hipEventRecord(ctx->eng_ev[buf], ctx->stream));
            if (ctx->eng_pending >= 0) {
                rc = process_chunk(ctx, ctx->eng_pending);
                if (rc) return rc;
            }
            ctx->eng_pending = buf;
            ctx->eng_next = buf ^ 1;
        } else {  // nothing left to advance: read the last chunk back
            rc = process_chunk(ctx, ctx->eng_pending);
            if (rc) return rc;
            ctx->eng_pending = -1;
        }
    }
    // results whose copies have landed; with nothing else in flight, wait for the rest
    bool idle = ctx->eng_pending < 0;
    for (const Slot& sl : ctx->slots) idle &= !sl.used;
    rc = collect_retired(ctx, idle, &completed);
    if (rc) return rc;
    if (n_done) *n_done = completed;
    return MDOT_OK;
}

int mdot_poll(mdot_ctx* ctx, uint64_t ticket, int wait, mdot_result* res)
{
    if (!ctx) return MDOT_E_ARG;
    for (;;) {
        auto it = ctx->finished.find(ticket);
        if (it != ctx->finished.end()) {
            if (res) *res = it->second;
            ctx->finished.erase(it);
            return MDOT_OK;
        }
        const Retiring* rt = nullptr;
        for (const Retiring& x : ctx->retiring)
            if (x.ticket == ticket) rt = &x;
        if (rt) {  // finished: its result lands with the copy queued at its retirement
            if (wait) HIPCHK(ctx, hipEventSynchronize(ctx->ret_ev[rt->hs]));
            int rc = collect_retired(ctx, false, nullptr);
            if (rc) return rc;
            if (!wait && !ctx->finished.count(ticket)) return 2;
            continue;
        }
        bool inflight = false;
        for (const Slot& sl : ctx->slots) inflight |= (sl.used && sl.ticket == ticket);
        if (!inflight) return fail(ctx, MDOT_E_ARG, "unknown ticket %llu", (unsigned long long)ticket);
        if (!wait) return 2;
        int rc = mdot_run(ctx, kBatchChunk, nullptr);
        if (rc) return rc;
    }
}

int mdot_inflight(mdot_ctx* ctx, int* n_active, size_t* bytes_in_use)
{
    if (!ctx) return MDOT_E_ARG;
    int rc = collect_retired(ctx, false, nullptr);
    if (rc) return rc;
    int a = (int)ctx->retiring.size();  // finished but their results not yet copied out
    for (const Slot& sl : ctx->slots) a += sl.used;
    if (n_active) *n_active = a;
    if (bytes_in_use) *bytes_in_use = ctx->bytes_in_use;
    return MDOT_OK;
}

}  // extern "C"
