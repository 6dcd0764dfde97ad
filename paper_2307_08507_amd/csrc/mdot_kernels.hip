// HIP kernels of the MDOT-PNCG hot path for gfx950 (MI355X).
//
// One solver step is two kernels on the context stream:
//   k_ctrl  : every workgroup reduces the per-block results of the previous sweep in a fixed
//             order and runs the scalar logic of the line search (App. B), PNCG (Alg. 2) and
//             the annealing loop (Alg. 1) on identical inputs, so all reach the same decision
//             without synchronising; each then applies the O(n) vector update for its slice
//             (accept a step, start a stage with smoothing + warm start, prepare Round), and
//             workgroup 0 stores the new state in the other state slot.
//   k_sweep : one fused O(n^2) pass over the cost: every workgroup forms
//             X_ij = u_i + v_j - gamma C_ij for a BR x BC tile (FP64 argument), takes one
//             exp per element and accumulates BOTH the row sums and the column sums from
//             that single read of C (row sums reduced across the wave64, column sums across
//             the four waves through LDS). The last workgroup of each row block / column
//             block combines the tile partials in FP64 (fixed order, so results do not
//             depend on scheduling) and reduces that block's contribution to the dot
//             products the next k_ctrl needs.
// The host never reads a value between steps; it replays a captured graph of steps and
// polls the done flag once per chunk.
//
// Exponent shifts: the row sum of row i is taken relative to a predicted log row sum s_i
// (the last accepted log r(P)_i moved by alpha p_i, or log r~_i at a stage start), so
// every exp argument of the entries that matter is O(1). Column sums reuse the same exp
// through per-row weights exp(s_i - S_I), S_I = max of s_i over the tile. A row or column
// whose shifted sum leaves [2^-64, 2^64] (FP32) is reported and the sweep is re-run with
// FP64 exp.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "mdot_internal.h"

namespace mdot {

#define LOG2E_D 1.4426950408889634074
#define LN2_D 0.6931471805599453094

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// ------------------------------------------------------------------ cost access
// Raw cost of row i at the lane's 4 consecutive columns j0..j0+3 (C = scale * raw).
// Columns >= n are returned as 0 and masked by the caller.
template <int DT>
struct DenseCost {
    const void* base;
    int n;
    bool vec;
    __device__ DenseCost(const Work& w) : base(w.cost), n(w.n), vec((w.n & 3) == 0) {}
    __device__ __forceinline__ void cols(int) {}
    __device__ __forceinline__ void row(int i, int j0, double c[4]) const
    {
        const size_t off = (size_t)i * n + j0;
        if constexpr (DT == MDOT_DT_F32) {
            const float* p = (const float*)base + off;
            if (vec && j0 + 3 < n) {
                float4 v = *(const float4*)p;
                c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = (j0 + k < n) ? (double)p[k] : 0.0;
            }
        } else if constexpr (DT == MDOT_DT_F64) {
            const double* p = (const double*)base + off;
            if (vec && j0 + 3 < n) {
                double2 a = *(const double2*)p;
                double2 b = *(const double2*)(p + 2);
                c[0] = a.x; c[1] = a.y; c[2] = b.x; c[3] = b.y;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = (j0 + k < n) ? p[k] : 0.0;
            }
        } else if constexpr (DT == MDOT_DT_F16) {
            const __half* p = (const __half*)base + off;
            if (vec && j0 + 3 < n) {
                uint2 raw = *(const uint2*)p;
                __half2 a = *(__half2*)&raw.x, b = *(__half2*)&raw.y;
                c[0] = __low2float(a); c[1] = __high2float(a); c[2] = __low2float(b); c[3] = __high2float(b);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = (j0 + k < n) ? (double)__half2float(p[k]) : 0.0;
            }
        } else {  // BF16
            const __hip_bfloat16* p = (const __hip_bfloat16*)base + off;
            if (vec && j0 + 3 < n) {
                uint2 raw = *(const uint2*)p;
                c[0] = __uint_as_float(raw.x << 16); c[1] = __uint_as_float(raw.x & 0xffff0000u);
                c[2] = __uint_as_float(raw.y << 16); c[3] = __uint_as_float(raw.y & 0xffff0000u);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = (j0 + k < n) ? (double)__bfloat162float(p[k]) : 0.0;
            }
        }
    }
};

// Point clouds: raw C_ij = sum_k (x_ik - y_jk)^2 (KIND 1) or sum_k |x_ik - y_jk| (KIND 2),
// evaluated in FP64 from FP32 coordinates (d <= 3).
template <int KIND>
struct PointCost {
    const float* X;
    const float* Y;
    int n, d;
    double y[4][3];
    __device__ PointCost(const Work& w) : X((const float*)w.cost), Y((const float*)w.cost + (size_t)w.n * w.d), n(w.n), d(w.d) {}
    __device__ __forceinline__ void cols(int j0)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int e = 0; e < 3; ++e) y[k][e] = (j0 + k < n && e < d) ? (double)Y[(size_t)(j0 + k) * d + e] : 0.0;
    }
    __device__ __forceinline__ void row(int i, int, double c[4]) const
    {
        double x[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) x[e] = (e < d) ? (double)X[(size_t)i * d + e] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                double t = x[e] - y[k][e];
                s = (KIND == 1) ? fma(t, t, s) : s + fabs(t);
            }
            c[k] = s;
        }
    }
};

// ------------------------------------------------------------------ tile bodies
struct TileCtx {
    int I, J, i0, j0lane, lane, wave, tid;
};

// Scalars a sweep needs from the state.
struct SweepArgs {
    double alpha, gamma, gamma_prev;
};

template <bool E64>
__device__ __forceinline__ double exp2_sel(double x)
{
    if constexpr (E64) return exp2(x);
    else return (double)__builtin_amdgcn_exp2f((float)x);
}

// Column combine: per-wave column values (4 per lane) -> one value per column of the tile.
__device__ __forceinline__ void col_combine_store(double* sbuf, const double v[4], const TileCtx& t, int op,
                                                  double* dst, int n, int jt0)
{
    // sbuf: [4 waves][kBC]
#pragma unroll
    for (int k = 0; k < 4; ++k) sbuf[t.wave * kBC + t.lane * 4 + k] = v[k];
    __syncthreads();
    {
        const int col = t.tid;  // kWG == kBC
        double a = sbuf[col], b = sbuf[kBC + col], c = sbuf[2 * kBC + col], d = sbuf[3 * kBC + col];
        double r = (op == 0) ? ((a + b) + (c + d)) : (op == 1 ? fmin(fmin(a, b), fmin(c, d)) : fmax(fmax(a, b), fmax(c, d)));
        if (jt0 + col < n) dst[jt0 + col] = r;
    }
    __syncthreads();
}

// LDS of one sweep workgroup: five per-row arrays and the per-wave column buffer.
constexpr int kSmem = 5 * kBR + 4 * kBC;

template <class Cost, bool E64>
__device__ void tile_lse(const Work& w, const SweepArgs& S, const TileCtx& t, int mode, double* sm)
{
    // mode SM_LSE: sums of exp; SM_MAX: maxima of X (FP64)
    double* sA = sm;
    double* sWt = sm + kBR;
    double* sS = sm + 2 * kBR;
    double* sCol = sm + 5 * kBR;
    const int n = w.n;
    const double alpha = S.alpha;
    const double g2 = S.gamma * w.scale * LOG2E_D;
    // per-row values: s_i (shift), A_i = (u_i - lz_i) log2 e, stored for the tile rows
    if (t.tid < kBR) {
        int i = t.i0 + t.tid;
        double s = -INFINITY, a = 0.0;
        if (i < n) {
            double ui = w.z[i], pi = w.p[i], li = w.lz[i];
            if (mode == SM_MAX) {
                a = (ui + alpha * pi) * LOG2E_D;
                s = 0.0;
            } else {
                s = li + alpha * pi;
                a = (ui - li) * LOG2E_D;
            }
        }
        sS[t.tid] = s;
        sA[t.tid] = a;
    }
    __syncthreads();
    // S_I = max_i s_i (identical in every workgroup of this row tile)
    double SI = -INFINITY;
    for (int k = 0; k < kBR; ++k) SI = fmax(SI, sS[k]);
    if (t.tid < kBR) sWt[t.tid] = (mode == SM_MAX) ? 1.0 : exp(sS[t.tid] - SI);
    __syncthreads();

    Cost cost(w);
    const int j0 = t.j0lane;
    cost.cols(j0);
    double V[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int j = j0 + k;
        ok[k] = j < n;
        V[k] = ok[k] ? (w.z[n + j] + alpha * w.p[n + j]) * LOG2E_D : 0.0;
    }
    double col64[4] = {0, 0, 0, 0};
    float col32[4] = {0, 0, 0, 0};
    double colmx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    const int rbase = t.wave * kRPW;
    for (int rr = 0; rr < kRPW; ++rr) {
        const int ir = rbase + rr;
        const int i = t.i0 + ir;
        if (i >= n) break;
        double c[4];
        cost.row(i, j0, c);
        const double A = sA[ir];
        if (mode == SM_MAX) {
            double m = -INFINITY;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double x = ok[k] ? fma(-g2, c[k], V[k]) + A : -INFINITY;  // log2 units
                m = fmax(m, x);
                colmx[k] = fmax(colmx[k], x);
            }
            m = wave_max(m);
            if (t.lane == 0) w.rowmin[(size_t)t.J * n + i] = m * LN2_D;
            continue;
        }
        if constexpr (E64) {
            const double wt = sWt[ir];
            double rs = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double e = ok[k] ? exp2(fma(-g2, c[k], V[k]) + A) : 0.0;
                rs += e;
                col64[k] = fma(wt, e, col64[k]);
            }
            rs = wave_sum(rs);
            if (t.lane == 0) w.rowpart[(size_t)t.J * n + i] = rs;
        } else {
            const float wt = (float)sWt[ir];
            float rs = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float e = ok[k] ? __builtin_amdgcn_exp2f((float)(fma(-g2, c[k], V[k]) + A)) : 0.f;
                rs += e;
                col32[k] = fmaf(wt, e, col32[k]);
            }
            double rsd = wave_sum((double)rs);
            if (t.lane == 0) w.rowpart[(size_t)t.J * n + i] = rsd;
            if ((rr & 7) == 7) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    col64[k] += (double)col32[k];
                    col32[k] = 0.f;
                }
            }
        }
    }
    if (mode == SM_MAX) {
        double out[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = colmx[k] * LN2_D;
        col_combine_store(sCol, out, t, 2, w.colmin + (size_t)t.I * n, n, t.J * kBC);
        return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) col64[k] += (double)col32[k];
    col_combine_store(sCol, col64, t, 0, w.colpart + (size_t)t.I * n, n, t.J * kBC);
    // every tile of row block I writes the same S_I, so the finalizer of any column block
    // reads it from one of the tiles it waited for
    if (t.tid == 0) w.tshift[t.I] = SI;
}

// Round pass 1 (Alg. 3, first half): column sums of F = D(x) P and the column c-transform
// g'_j = min_i (C_ij - f_i); also the row c-transform f''_i = min_j (C_ij - g_j), for the
// two potential sets (u, v)/gamma and their finite differences along the annealing path.
template <class Cost, bool E64>
__device__ void tile_r1(const Work& w, const SweepArgs& S, const TileCtx& t, double* sm)
{
    double* sA = sm;
    double* sWt = sm + kBR;
    double* sS = sm + 2 * kBR;
    double* sF1 = sm + 3 * kBR;
    double* sF2 = sm + 4 * kBR;
    double* sCol = sm + 5 * kBR;
    const int n = w.n;
    const double g2 = S.gamma * w.scale * LOG2E_D;
    const double inv_g = 1.0 / S.gamma;
    const double dg = S.gamma - S.gamma_prev;
    const bool ext = dg > 0.0;
    const double inv_dg = ext ? 1.0 / dg : 0.0;
    if (t.tid < kBR) {
        int i = t.i0 + t.tid;
        double s = -INFINITY, a = 0.0, f1 = INFINITY, f2 = INFINITY;
        if (i < n) {
            double ui = w.z[i], li = w.lz[i];
            s = li;
            a = (ui - li) * LOG2E_D;
            f1 = ui * inv_g;
            f2 = ext ? (ui - w.zprev[i]) * inv_dg : f1;
        }
        sS[t.tid] = s; sA[t.tid] = a; sF1[t.tid] = f1; sF2[t.tid] = f2;
    }
    __syncthreads();
    double SI = -INFINITY;
    for (int k = 0; k < kBR; ++k) SI = fmax(SI, sS[k]);
    if (t.tid < kBR) {
        int i = t.i0 + t.tid;
        sWt[t.tid] = (i < n) ? exp(sS[t.tid] - SI) * w.xr[i] : 0.0;
    }
    __syncthreads();
    Cost cost(w);
    const int j0 = t.j0lane;
    cost.cols(j0);
    double V[4], G1[4], G2[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int j = j0 + k;
        ok[k] = j < n;
        double vj = ok[k] ? w.z[n + j] : 0.0;
        V[k] = vj * LOG2E_D;
        G1[k] = ok[k] ? vj * inv_g : INFINITY;
        G2[k] = ok[k] ? (ext ? (vj - w.zprev[n + j]) * inv_dg : vj * inv_g) : INFINITY;
    }
    double col64[4] = {0, 0, 0, 0};
    double cm1[4] = {INFINITY, INFINITY, INFINITY, INFINITY}, cm2[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    const double sc = w.scale;
    const int rbase = t.wave * kRPW;
    for (int rr = 0; rr < kRPW; ++rr) {
        const int ir = rbase + rr;
        const int i = t.i0 + ir;
        if (i >= n) break;
        double c[4];
        cost.row(i, j0, c);
        const double A = sA[ir], wt = sWt[ir], f1 = sF1[ir], f2 = sF2[ir];
        double rm1 = INFINITY, rm2 = INFINITY;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k]) continue;
            double e = exp2_sel<E64>(fma(-g2, c[k], V[k]) + A);
            col64[k] = fma(wt, e, col64[k]);
            double cv = sc * c[k];
            cm1[k] = fmin(cm1[k], cv - f1);
            cm2[k] = fmin(cm2[k], cv - f2);
            rm1 = fmin(rm1, cv - G1[k]);
            rm2 = fmin(rm2, cv - G2[k]);
        }
        rm1 = wave_min(rm1);
        rm2 = wave_min(rm2);
        if (t.lane == 0) {
            w.rowmin[(size_t)t.J * n + i] = rm1;
            w.rowmin[(size_t)(w.nct + t.J) * n + i] = rm2;
        }
    }
    col_combine_store(sCol, col64, t, 0, w.colpart + (size_t)t.I * n, n, t.J * kBC);
    col_combine_store(sCol, cm1, t, 1, w.colmin + (size_t)t.I * n, n, t.J * kBC);
    col_combine_store(sCol, cm2, t, 1, w.colmin + (size_t)(w.nrt + t.I) * n, n, t.J * kBC);
    // every tile of row block I writes the same S_I, so the finalizer of any column block
    // reads it from one of the tiles it waited for
    if (t.tid == 0) w.tshift[t.I] = SI;
}

// Round pass 2: row sums of F' = D(x) P D(y): r(F')_i and sum_j F'_ij C_ij; (C err_c)_i;
// the row c-transform f'_i = min_j (C_ij - g'_j) and the column c-transform
// g''_j = min_i (C_ij - f''_i) (both potential sets).
template <class Cost, bool E64>
__device__ void tile_r2(const Work& w, const SweepArgs& S, const TileCtx& t, double* sm)
{
    double* sA = sm;
    double* sF1 = sm + 3 * kBR;
    double* sF2 = sm + 4 * kBR;
    double* sCol = sm + 5 * kBR;
    const int n = w.n;
    const double g2 = S.gamma * w.scale * LOG2E_D;
    if (t.tid < kBR) {
        int i = t.i0 + t.tid;
        double a = 0.0, f1 = INFINITY, f2 = INFINITY;
        if (i < n) {
            a = (w.z[i] - w.lz[i]) * LOG2E_D;
            f1 = w.fpp[i];
            f2 = w.fpp[n + i];
        }
        sA[t.tid] = a; sF1[t.tid] = f1; sF2[t.tid] = f2;
    }
    __syncthreads();
    Cost cost(w);
    const int j0 = t.j0lane;
    cost.cols(j0);
    // V is the same as in pass 1, so every exp below is bit-identical to pass 1's and the
    // implicit plan F' = D(x) P D(y) is one matrix across both passes; y is applied in FP64.
    double V[4], Y[4], GP1[4], GP2[4], EC[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int j = j0 + k;
        ok[k] = j < n;
        Y[k] = ok[k] ? w.yc[j] : 0.0;
        V[k] = ok[k] ? w.z[n + j] * LOG2E_D : 0.0;
        GP1[k] = ok[k] ? w.gp[j] : INFINITY;
        GP2[k] = ok[k] ? w.gp[n + j] : INFINITY;
        EC[k] = ok[k] ? w.errc[j] : 0.0;
    }
    double cm1[4] = {INFINITY, INFINITY, INFINITY, INFINITY}, cm2[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    const double sc = w.scale;
    const int rbase = t.wave * kRPW;
    for (int rr = 0; rr < kRPW; ++rr) {
        const int ir = rbase + rr;
        const int i = t.i0 + ir;
        if (i >= n) break;
        double c[4];
        cost.row(i, j0, c);
        const double A = sA[ir], f1 = sF1[ir], f2 = sF2[ir];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, rm1 = INFINITY, rm2 = INFINITY;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k]) continue;
            double cv = sc * c[k];
            double e = exp2_sel<E64>(fma(-g2, c[k], V[k]) + A) * Y[k];
            s0 += e;
            s1 = fma(e, cv, s1);
            s2 = fma(cv, EC[k], s2);
            rm1 = fmin(rm1, cv - GP1[k]);
            rm2 = fmin(rm2, cv - GP2[k]);
            cm1[k] = fmin(cm1[k], cv - f1);
            cm2[k] = fmin(cm2[k], cv - f2);
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        rm1 = wave_min(rm1);
        rm2 = wave_min(rm2);
        if (t.lane == 0) {
            const size_t o = (size_t)t.J * n + i;
            w.rowpart[o] = s0;
            w.rowpart2[o] = s1;
            w.rowpart3[o] = s2;
            w.rowmin[o] = rm1;
            w.rowmin[(size_t)(w.nct + t.J) * n + i] = rm2;
        }
    }
    col_combine_store(sCol, cm1, t, 1, w.colmin + (size_t)t.I * n, n, t.J * kBC);
    col_combine_store(sCol, cm2, t, 1, w.colmin + (size_t)(w.nrt + t.I) * n, n, t.J * kBC);
}

// ------------------------------------------------------------------ finalizers
// Block reduction of kNDot values (fixed tree). sred: LDS of kNDot * 4 doubles.
__device__ void block_dots(double v[kNDot], double* dst, int tid, double* sred)
{
#pragma unroll
    for (int d = 0; d < kNDot; ++d) {
        double s = wave_sum(v[d]);
        if ((tid & 63) == 0) sred[d * 4 + (tid >> 6)] = s;
    }
    __syncthreads();
    if (tid < kNDot) dst[tid] = (sred[tid * 4 + 0] + sred[tid * 4 + 1]) + (sred[tid * 4 + 2] + sred[tid * 4 + 3]);
    __syncthreads();
}

__device__ __forceinline__ bool in_range(double s, bool e64)
{
    const double lo = e64 ? 0x1p-900 : 0x1p-64, hi = e64 ? 0x1p900 : 0x1p64;
    return s >= lo && s <= hi;  // false for NaN
}

// Rows i0 .. i0+kBR-1 of row block I.
__device__ void finalize_rows(const Work& w, const SweepArgs& S, int I, int tid, bool e64, int mode, double* sred)
{
    const int n = w.n;
    const int i = I * kBR + (tid >> 2);
    const int q = tid & 3;  // 4 threads per row share the column tiles
    const bool live = i < n;
    double v[kNDot];
#pragma unroll
    for (int d = 0; d < kNDot; ++d) v[d] = 0.0;
    if (mode == SM_MAX) {
        double m = -INFINITY;
        if (live)
            for (int J = q; J < w.nct; J += 4) m = fmax(m, w.rowmin[(size_t)J * n + i]);
        m = fmax(m, __shfl_xor(m, 1, 64));
        m = fmax(m, __shfl_xor(m, 2, 64));
        if (live && q == 0) w.lz[i] = m;
        block_dots(v, w.bdots + (size_t)I * kNDot, tid, sred);
        return;
    }
    if (mode == SM_LSE) {
        double s = 0.0;
        if (live)
            for (int J = q; J < w.nct; J += 4) s += w.rowpart[(size_t)J * n + i];
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        if (live && q == 0) {
            const double pi = w.p[i];
            const double sh = w.lz[i] + S.alpha * pi;
            const double l = sh + log(s);
            w.lzt[i] = l;
            const double gnew = exp(l) - w.rt[i];
            const double snew = w.logt[i] - l;
            const double y = gnew - w.g[i];
            v[D_PHI] = pi * gnew;
            v[D_NUM] = -y * snew;
            v[D_DEN] = y * pi;
            v[D_SG] = snew * gnew;
            v[D_GN] = fabs(gnew);
            v[D_BAD] = in_range(s, e64) ? 0.0 : 1.0;
        }
    } else if (mode == SM_R1) {
        double m1 = INFINITY, m2 = INFINITY;
        if (live)
            for (int J = q; J < w.nct; J += 4) {
                m1 = fmin(m1, w.rowmin[(size_t)J * n + i]);
                m2 = fmin(m2, w.rowmin[(size_t)(w.nct + J) * n + i]);
            }
        m1 = fmin(m1, __shfl_xor(m1, 1, 64)); m1 = fmin(m1, __shfl_xor(m1, 2, 64));
        m2 = fmin(m2, __shfl_xor(m2, 1, 64)); m2 = fmin(m2, __shfl_xor(m2, 2, 64));
        if (live && q == 0) {
            w.fpp[i] = m1;
            w.fpp[n + i] = m2;
            v[D_RF1] = w.r[i] * m1;
            v[D_RF2] = w.r[i] * m2;
        }
    } else {  // SM_R2
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, m1 = INFINITY, m2 = INFINITY;
        if (live)
            for (int J = q; J < w.nct; J += 4) {
                const size_t o = (size_t)J * n + i;
                s0 += w.rowpart[o];
                s1 += w.rowpart2[o];
                s2 += w.rowpart3[o];
                m1 = fmin(m1, w.rowmin[o]);
                m2 = fmin(m2, w.rowmin[(size_t)(w.nct + J) * n + i]);
            }
#pragma unroll
        for (int o = 1; o <= 2; o <<= 1) {
            s0 += __shfl_xor(s0, o, 64);
            s1 += __shfl_xor(s1, o, 64);
            s2 += __shfl_xor(s2, o, 64);
            m1 = fmin(m1, __shfl_xor(m1, o, 64));
            m2 = fmin(m2, __shfl_xor(m2, o, 64));
        }
        if (live && q == 0) {
            const double ex = w.xr[i] * exp(w.lz[i]);
            const double rF = ex * s0;             // r(F')_i
            const double er = w.r[i] - rF;         // err_r
            v[D_A] = ex * s1;
            v[D_ERRR] = er;
            v[D_EC] = er * s2;
            v[D_RFP1] = w.r[i] * m1;
            v[D_RFP2] = w.r[i] * m2;
        }
    }
    block_dots(v, w.bdots + (size_t)I * kNDot, tid, sred);
}

// Columns of column block J (one thread per column).
__device__ void finalize_cols(const Work& w, const SweepArgs& S, int J, int tid, bool e64, int mode, double* sm,
                              double* sred)
{
    double* sfac = sm;  // [nrt] (nrt <= 1024 < kSmem)
    double* pM = sm + 1300;
    const int n = w.n;
    const int j = J * kBC + tid;
    const bool live = j < n;
    double v[kNDot];
#pragma unroll
    for (int d = 0; d < kNDot; ++d) v[d] = 0.0;
    if (mode == SM_MAX) {
        double m = -INFINITY;
        if (live)
            for (int I = 0; I < w.nrt; ++I) m = fmax(m, w.colmin[(size_t)I * n + j]);
        if (live) w.lz[n + j] = m;
        block_dots(v, w.bdots + (size_t)(w.nrt + J) * kNDot, tid, sred);
        return;
    }
    if (mode == SM_LSE || mode == SM_R1) {
        // combine tile partials taken relative to S_I
        if (tid == 0) {
            double M = -INFINITY;
            for (int I = 0; I < w.nrt; ++I) M = fmax(M, w.tshift[I]);
            *pM = M;
        }
        __syncthreads();
        const double M = *pM;
        for (int I = tid; I < w.nrt; I += kWG) sfac[I] = exp(w.tshift[I] - M);
        __syncthreads();
        double s = 0.0;
        if (live)
            for (int I = 0; I < w.nrt; ++I) s = fma(w.colpart[(size_t)I * n + j], sfac[I], s);
        if (mode == SM_LSE) {
            if (live) {
                const double pj = w.p[n + j];
                const double l = M + log(s);
                w.lzt[n + j] = l;
                const double gnew = exp(l) - w.rt[n + j];
                const double snew = w.logt[n + j] - l;
                const double y = gnew - w.g[n + j];
                v[D_PHI] = pj * gnew;
                v[D_NUM] = -y * snew;
                v[D_DEN] = y * pj;
                v[D_SG] = snew * gnew;
                v[D_GN] = fabs(gnew);
                v[D_BAD] = in_range(s, e64) ? 0.0 : 1.0;
            }
        } else {  // R1: c(F)_j, y_j, err_c, g'_j
            double m1 = INFINITY, m2 = INFINITY;
            if (live)
                for (int I = 0; I < w.nrt; ++I) {
                    m1 = fmin(m1, w.colmin[(size_t)I * n + j]);
                    m2 = fmin(m2, w.colmin[(size_t)(w.nrt + I) * n + j]);
                }
            if (live) {
                const double cF = exp(M) * s;
                const double cj = w.c[j];
                const double y = (cF > 0.0) ? fmin(cj / cF, 1.0) : 1.0;
                const double ec = cj - y * cF;
                w.yc[j] = y;
                w.errc[j] = ec;
                w.gp[j] = m1;
                w.gp[n + j] = m2;
                v[D_CG1] = cj * m1;
                v[D_CG2] = cj * m2;
                v[D_ERRC] = ec;
            }
        }
    } else {  // R2: g''_j
        double m1 = INFINITY, m2 = INFINITY;
        if (live)
            for (int I = 0; I < w.nrt; ++I) {
                m1 = fmin(m1, w.colmin[(size_t)I * n + j]);
                m2 = fmin(m2, w.colmin[(size_t)(w.nrt + I) * n + j]);
            }
        if (live) {
            v[D_CGP1] = w.c[j] * m1;
            v[D_CGP2] = w.c[j] * m2;
        }
    }
    block_dots(v, w.bdots + (size_t)(w.nrt + J) * kNDot, tid, sred);
}

// ------------------------------------------------------------------ scalar state machine
__device__ __forceinline__ void next_stage(State& S, const DevParams& P)
{
    const double gnew = fmin(S.gamma + (P.q - 1.0) * S.gamma, P.gamma_f);  // Alg. 1
    const double dg = gnew - S.gamma, dgp = S.gamma - S.gamma_prev;
    S.ws_ratio = P.warm_start ? dg / dgp : 0.0;  // eq. (approx-znext)
    S.gamma_prev = S.gamma;
    S.gamma = gnew;
    S.stage += 1;
    S.eps_d = P.hmin / pow(gnew, P.p);  // entropy-aware tolerance
    S.w = fmin(S.eps_d / 4.0, 0.5);     // variable smoothing weight
    S.tol = fmax(S.eps_d / 2.0, P.tol_floor);
    // precision ladder: FP32 exp while the tolerance is far above FP32 resolution
    S.exp64_stage = P.exp64_default || S.tol < P.f32_min_tol;
    S.exp64 = S.exp64_stage;
    S.alpha_prev = 1.0;
    S.vec_action |= VA_STAGE_INIT;
    S.sweep_mode = SM_LSE;
    S.ls_phase = LS_INIT;
}

__device__ __forceinline__ void end_stage(State& S, const DevParams& P, bool converged)
{
    if (!converged) S.inner_warn = 1;
    if (P.adaptive || S.gamma >= P.gamma_f || S.budget_stop) {
        S.vec_action |= VA_ROUND_PREP;
        S.sweep_mode = SM_R1;
    } else {
        next_stage(S, P);
    }
}

__device__ __forceinline__ void finish(State& S, int status)
{
    S.done = 1;
    S.status = status;
    S.sweep_mode = SM_NONE;
}

__device__ __forceinline__ void start_line_search(State& S)
{
    S.ls_phase = LS_TRIAL;
    S.alpha = S.alpha_prev;
    S.alo = 0.0;
    S.dlo = S.dphi0;
    S.ahi = INFINITY;
    S.dhi = 0.0;
    S.ls_trials_cur = 0;
}

// Scalar logic after a sweep: line search (App. B), PNCG bookkeeping (Alg. 2), stage
// control (Alg. 1) and the certified-gap termination. `sum` holds the global dots.
__device__ __forceinline__ void decide(State& S, const DevParams& P, const double* sum)
{
    const int mode = S.sweep_mode;
    S.vec_action = 0;
    if (mode == SM_MAX) {  // standalone LSE: the row maxima become the row shifts
        S.sweep_mode = SM_LSE;
        return;
    }
    if (mode == SM_LSE) {
        const bool bad = sum[D_BAD] > 0.0;
        if (bad && !S.exp64) {  // re-run this sweep with FP64 exp
            S.exp64 = 1;
            S.fallbacks++;
            return;
        }
        S.exp64 = S.exp64_stage;
        if (S.standalone) {
            if (bad) S.status = MDOT_W_RANGE;
            if (S.standalone == 2) {  // round-and-certify: lzt -> lz, then Round
                S.alpha_acc = 0.0;
                S.beta = 0.0;
                S.reset = 1;
                S.vec_action = VA_ACCEPT | VA_ROUND_PREP;
                S.sweep_mode = SM_R1;
            } else {
                finish(S, S.status);
            }
            return;
        }
        S.sweeps++;
        if (P.max_sweeps > 0 && S.sweeps >= P.max_sweeps) S.budget_stop = 1;
        const double gn = sum[D_GN], sg = sum[D_SG];
        const double d = bad ? NAN : sum[D_PHI];
        if (S.ls_phase == LS_INIT) {  // first sweep of a stage: p = s, beta = 0
            S.alpha_acc = 0.0;
            S.beta = 0.0;
            S.reset = 1;
            S.vec_action = VA_ACCEPT;
            S.gnorm = gn;
            S.k = 1;
            S.dphi0 = sg;
            if (gn <= S.tol) end_stage(S, P, true);
            else if (!(sg < 0.0) || S.budget_stop) end_stage(S, P, false);
            else start_line_search(S);
            return;
        }
        bool accept;
        if (S.ls_phase == LS_FORCE) {
            accept = true;
        } else {
            S.ls_trials++;
            S.ls_trials_cur++;
            accept = ((2.0 * P.c1 - 1.0) * S.dphi0 >= d) && (d >= P.c2 * S.dphi0);  // eq. (approximate-wolfe)
        }
        if (accept) {
            const double num = sum[D_NUM], den = sum[D_DEN];
            const double beta = (den != 0.0) ? num / den : 0.0;  // eq. (beta_PPR_OT)
            double pg = sg + beta * sum[D_PHI];                  // <s + beta p, g_new>
            const int reset = !(pg < 0.0);
            if (reset) {  // not a descent direction: restart with s (Alg. 2)
                pg = sg;
                S.cg_resets++;
            }
            S.alpha_acc = S.alpha;
            S.alpha_prev = S.alpha;
            S.beta = beta;
            S.reset = reset;
            S.vec_action = VA_ACCEPT;
            S.pncg_iters++;
            S.k++;
            S.gnorm = gn;
            S.dphi0 = pg;
            if (gn <= S.tol) end_stage(S, P, true);
            else if (S.k > P.max_pncg_iters || S.budget_stop || !(pg < 0.0)) end_stage(S, P, false);
            else start_line_search(S);
            return;
        }
        // not accepted: shrink the bracket [alpha_lo, alpha_hi] with phi'(lo) < 0 < phi'(hi)
        if (d < 0.0) {
            S.alo = S.alpha;
            S.dlo = d;
        } else {  // NaN (range failure in FP64 too) also lands here: step too long
            S.ahi = S.alpha;
            S.dhi = d;
        }
        if (S.budget_stop) {  // stop at the last accepted iterate
            end_stage(S, P, false);
            return;
        }
        if (isinf(S.ahi)) {
            S.alpha = 2.0 * S.alpha;
        } else {  // hybrid step: mean of the secant point and the bisection point
            double asec = (S.alo * S.dhi - S.ahi * S.dlo) / (S.dhi - S.dlo);
            const double amid = 0.5 * (S.alo + S.ahi);
            if (!(asec > S.alo && asec < S.ahi)) asec = amid;
            S.alpha = 0.5 * asec + 0.5 * amid;
        }
        if (S.ls_trials_cur >= P.max_ls_trials) {
            S.ls_failures++;
            if (S.alo > 0.0) {
                S.alpha = S.alo;
                S.ls_phase = LS_FORCE;
            } else {
                end_stage(S, P, false);
            }
        }
        return;
    }
    if (mode == SM_R1) {
        S.cert_sweeps++;
        S.r1[0] = sum[D_CG1];
        S.r1[1] = sum[D_CG2];
        S.r1[2] = sum[D_RF1];
        S.r1[3] = sum[D_RF2];
        S.errc_sum = sum[D_ERRC];
        S.sweep_mode = SM_R2;
        return;
    }
    // SM_R2: UB = <G, C> with G = F' + err_r err_c^T / ||err_r||_1 (Alg. 3), LB, termination
    S.cert_sweeps++;
    const double L = sum[D_ERRR];
    const double ub = sum[D_A] + (L > 0.0 ? sum[D_EC] / L : 0.0);
    const double lb = fmax(fmax(S.r1[0] + sum[D_RFP1], S.r1[1] + sum[D_RFP2]),
                           fmax(S.r1[2] + sum[D_CGP1], S.r1[3] + sum[D_CGP2]));
    const double me = fabs(S.errc_sum - L);
    S.last_ub = ub;
    S.last_lb = lb;
    if (S.standalone) {
        S.best_ub = ub;
        S.best_lb = lb;
        S.best_me = me;
        finish(S, S.status);
        return;
    }
    if (ub < S.best_ub) {
        S.best_ub = ub;
        S.best_gamma = S.gamma;
        S.best_me = me;
        S.vec_action |= VA_SAVE_BEST;
    }
    if (lb > S.best_lb) S.best_lb = lb;
    if (P.adaptive && S.best_ub - S.best_lb <= P.target) finish(S, MDOT_OK);
    else if (S.budget_stop) finish(S, MDOT_W_NOT_CONVERGED);
    else if (S.gamma >= P.gamma_f) finish(S, (P.adaptive || S.inner_warn) ? MDOT_W_NOT_CONVERGED : MDOT_OK);
    else next_stage(S, P);
}

// ------------------------------------------------------------------ the sweep kernel
template <bool E64, bool ROUND>
__device__ __forceinline__ void sweep_tiles(const Work& w, const SweepArgs& a, const TileCtx& t, int mode, double* smem)
{
#define MDOT_DISPATCH(COST)                                                  \
    do {                                                                     \
        if constexpr (!ROUND) tile_lse<COST, E64>(w, a, t, mode, smem);      \
        else if (mode == SM_R1) tile_r1<COST, E64>(w, a, t, smem);           \
        else tile_r2<COST, E64>(w, a, t, smem);                              \
    } while (0)
    if (w.cost_kind == MDOT_COST_DENSE) {
        switch (w.dtype) {
            case MDOT_DT_F32: MDOT_DISPATCH(DenseCost<MDOT_DT_F32>); break;
            case MDOT_DT_F64: MDOT_DISPATCH(DenseCost<MDOT_DT_F64>); break;
            case MDOT_DT_F16: MDOT_DISPATCH(DenseCost<MDOT_DT_F16>); break;
            default: MDOT_DISPATCH(DenseCost<MDOT_DT_BF16>); break;
        }
    } else if (w.cost_kind == MDOT_COST_POINTS_SQEUCLID) {
        MDOT_DISPATCH(PointCost<1>);
    } else {
        MDOT_DISPATCH(PointCost<2>);
    }
#undef MDOT_DISPATCH
}

// Shared body of the two sweep kernels. ROUND = false: LSE and max sweeps (the hot path);
// ROUND = true: the two Round/certificate sweeps, kept in their own kernel so their larger
// register footprint does not lower the occupancy of the LSE sweep.
template <bool ROUND>
__device__ __forceinline__ void sweep_kernel_body(const Work& w, int parity)
{
    __shared__ double smem[kSmem];
    __shared__ double sred[kNDot * 4];
    __shared__ int sflag[2];
    const State* Sp = w.st + (parity ^ 1);  // written by this step's control kernel
    const int mode = Sp->sweep_mode;
    if (mode == SM_NONE || Sp->done) return;
    if ((mode == SM_R1 || mode == SM_R2) != ROUND) return;
    const bool e64 = Sp->exp64 != 0;
    const int ph = Sp->ls_phase;
    SweepArgs a;
    a.alpha = (mode == SM_LSE && (ph == LS_TRIAL || ph == LS_FORCE)) ? Sp->alpha : 0.0;
    a.gamma = Sp->gamma;
    a.gamma_prev = Sp->gamma_prev;
    TileCtx t;
    t.tid = threadIdx.x;
    t.lane = t.tid & 63;
    t.wave = t.tid >> 6;
    t.I = blockIdx.x / w.nct;
    t.J = blockIdx.x % w.nct;
    t.i0 = t.I * kBR;
    t.j0lane = t.J * kBC + t.lane * 4;
    if (e64) sweep_tiles<true, ROUND>(w, a, t, mode, smem);
    else sweep_tiles<false, ROUND>(w, a, t, mode, smem);

    // arrival: the last tile of row block I / column block J finalizes it
    __threadfence();
    __syncthreads();
    if (t.tid == 0) {
        uint32_t x = __hip_atomic_fetch_add(&w.cnt[t.I], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t y = __hip_atomic_fetch_add(&w.cnt[w.nrt + t.J], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sflag[0] = (x == (uint32_t)w.nct - 1);
        sflag[1] = (y == (uint32_t)w.nrt - 1);
    }
    __syncthreads();
    const bool lastR = sflag[0], lastC = sflag[1];
    if (!lastR && !lastC) return;
    __threadfence();
    if (lastR) {
        finalize_rows(w, a, t.I, t.tid, e64, mode, sred);
        if (t.tid == 0) w.cnt[t.I] = 0;
    }
    if (lastC) {
        finalize_cols(w, a, t.J, t.tid, e64, mode, smem, sred);
        if (t.tid == 0) w.cnt[w.nrt + t.J] = 0;
    }
}

__global__ void __launch_bounds__(kWG) k_sweep(const Work* __restrict__ wp, int parity)
{
    sweep_kernel_body<false>(*wp, parity);
}

__global__ void __launch_bounds__(kWG) k_round(const Work* __restrict__ wp, int parity)
{
    sweep_kernel_body<true>(*wp, parity);
}

// ------------------------------------------------------------------ the control kernel
__global__ void __launch_bounds__(kVecWG) k_ctrl(const Work* __restrict__ wp, int parity)
{
    __shared__ double sred[kNDot * 4];
    __shared__ double sglob[kNDot];
    __shared__ double sf[8];
    __shared__ int si[4];
    const Work w = *wp;
    const int tid = threadIdx.x;
    // fixed-order reduction of the previous sweep's block results (identical in every WG)
    const int nb = w.nrt + w.nct;
    double v[kNDot];
#pragma unroll
    for (int d = 0; d < kNDot; ++d) v[d] = 0.0;
    for (int b = tid; b < nb; b += kVecWG)
#pragma unroll
        for (int d = 0; d < kNDot; ++d) v[d] += w.bdots[(size_t)b * kNDot + d];
    block_dots(v, sglob, tid, sred);
    if (tid == 0) {
        State S = w.st[parity];
        const DevParams P = *w.prm;
        if (S.pending && !S.done) {
            double sum[kNDot];
#pragma unroll
            for (int d = 0; d < kNDot; ++d) sum[d] = sglob[d];
            decide(S, P, sum);
        }
        si[0] = S.vec_action;
        si[1] = S.reset;
        si[2] = S.stage;
        sf[0] = S.alpha_acc;
        sf[1] = S.beta;
        sf[2] = S.w;
        sf[3] = S.ws_ratio;
        S.vec_action = 0;
        S.pending = (S.sweep_mode != SM_NONE && !S.done);
        if (blockIdx.x == 0) w.st[parity ^ 1] = S;
    }
    __syncthreads();
    const int va = si[0];
    if (va == 0) return;
    const int n = w.n;
    const int k = blockIdx.x * blockDim.x + tid;
    if (k >= 2 * n) return;
    double zk = w.z[k];
    if (va & VA_ACCEPT) {  // (u, v) += alpha p; new direction p = s + beta p, or s on reset (Alg. 2)
        zk = fma(sf[0], w.p[k], zk);
        w.z[k] = zk;
        const double l = w.lzt[k];
        w.lz[k] = l;
        w.g[k] = exp(l) - w.rt[k];
        const double sdir = w.logt[k] - l;  // Sinkhorn direction, eq. (sinkhorn-direction)
        w.p[k] = si[1] ? sdir : fma(sf[1], w.p[k], sdir);
    }
    if (va & VA_SAVE_BEST) w.zbest[k] = zk;
    if (va & VA_STAGE_INIT) {  // Alg. 1: smoothing, rank-1 start or warm start eq. (approx-znext)
        const double m = (k < n) ? w.r[k] : w.c[k - n];
        const double rt = (1.0 - sf[2]) * m + sf[2] / n;
        const double lt = log(rt);
        w.rt[k] = rt;
        w.logt[k] = lt;
        if (si[2] == 1) {
            zk = lt;
            w.zprev[k] = lt;  // z^0 at gamma^0 = 0
        } else {
            const double zp = w.zprev[k];
            w.zprev[k] = zk;
            zk = zk + sf[3] * (zk - zp);
        }
        w.z[k] = zk;
        w.p[k] = 0.0;
        w.g[k] = 0.0;
        w.lz[k] = lt;  // predicted log marginals of the warm-started plan (row shifts)
    }
    if ((va & VA_ROUND_PREP) && k < n) {  // Alg. 3: x = r / r(P) ^ 1
        const double rp = exp(w.lz[k]);
        w.xr[k] = (rp > 0.0) ? fmin(w.r[k] / rp, 1.0) : 1.0;
    }
}

// ------------------------------------------------------------------ set-up kernels
__global__ void k_init(const Work* __restrict__ wp)
{
    const Work w = *wp;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const DevParams P = *w.prm;
    State S;
    memset(&S, 0, sizeof(S));
    S.stage = 1;
    S.gamma = fmin(P.gamma_i, P.gamma_f);
    S.gamma_prev = 0.0;
    S.eps_d = P.hmin / pow(S.gamma, P.p);
    S.w = fmin(S.eps_d / 4.0, 0.5);
    S.tol = fmax(S.eps_d / 2.0, P.tol_floor);
    S.exp64_stage = P.exp64_default || S.tol < P.f32_min_tol;
    S.exp64 = S.exp64_stage;
    S.alpha_prev = 1.0;
    S.vec_action = VA_STAGE_INIT;
    S.sweep_mode = SM_LSE;
    S.ls_phase = LS_INIT;
    S.best_ub = INFINITY;
    S.best_lb = -INFINITY;
    S.best_gamma = S.gamma;
    S.pending = 0;
    w.st[0] = S;
    w.st[1] = S;
    for (int k = 0; k < w.nrt + w.nct; ++k) w.cnt[k] = 0;
}

// Intake statistics: out8 = {sum r, sum c, min r, min c, H(r), H(c), nonfinite count, 0}
__global__ void k_intake(const Work* __restrict__ wp, double* out8)
{
    const Work w = *wp;
    __shared__ double sred[8][kWG];
    const int n = w.n, t = threadIdx.x;
    double sr = 0, sc = 0, mr = INFINITY, mc = INFINITY, hr = 0, hc = 0, bad = 0;
    for (int i = t; i < n; i += kWG) {
        double a = w.r[i], b = w.c[i];
        if (!isfinite(a) || !isfinite(b)) bad += 1;
        sr += a; sc += b;
        mr = fmin(mr, a); mc = fmin(mc, b);
        if (a > 0) hr -= a * log(a);
        if (b > 0) hc -= b * log(b);
    }
    sred[0][t] = sr; sred[1][t] = sc; sred[2][t] = mr; sred[3][t] = mc;
    sred[4][t] = hr; sred[5][t] = hc; sred[6][t] = bad; sred[7][t] = 0;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (t < h) {
            for (int d = 0; d < 8; ++d) {
                if (d == 2 || d == 3) sred[d][t] = fmin(sred[d][t], sred[d][t + h]);
                else sred[d][t] += sred[d][t + h];
            }
        }
        __syncthreads();
    }
    if (t < 8) out8[t] = sred[t][0];
}

// Cost range over a dense matrix or the maximum raw point distance: out2 = {min, max} of raw
// values (non-finite entries make max NaN).
template <class Cost>
__device__ void cost_range_body(const Work& w, double* mn, double* mx)
{
    const int n = w.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int I = blockIdx.x / w.nct, J = blockIdx.x % w.nct;
    const int j0 = J * kBC + lane * 4;
    Cost cost(w);
    cost.cols(j0);
    double lo = INFINITY, hi = -INFINITY;
    for (int rr = 0; rr < kRPW; ++rr) {
        const int i = I * kBR + wave * kRPW + rr;
        if (i >= n) break;
        double c[4];
        cost.row(i, j0, c);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (j0 + k < n) {
                if (!isfinite(c[k])) hi = NAN;
                lo = fmin(lo, c[k]);
                hi = (hi != hi) ? hi : fmax(hi, c[k]);
            }
    }
    *mn = lo;
    *mx = hi;
}

__global__ void __launch_bounds__(kWG) k_cost_range(const Work* __restrict__ wp, double* part)
{
    const Work w = *wp;
    double lo, hi;
    if (w.cost_kind == MDOT_COST_DENSE) {
        switch (w.dtype) {
            case MDOT_DT_F32: cost_range_body<DenseCost<MDOT_DT_F32>>(w, &lo, &hi); break;
            case MDOT_DT_F64: cost_range_body<DenseCost<MDOT_DT_F64>>(w, &lo, &hi); break;
            case MDOT_DT_F16: cost_range_body<DenseCost<MDOT_DT_F16>>(w, &lo, &hi); break;
            default: cost_range_body<DenseCost<MDOT_DT_BF16>>(w, &lo, &hi); break;
        }
    } else if (w.cost_kind == MDOT_COST_POINTS_SQEUCLID) {
        cost_range_body<PointCost<1>>(w, &lo, &hi);
    } else {
        cost_range_body<PointCost<2>>(w, &lo, &hi);
    }
    __shared__ double s0[kWG], s1[kWG];
    const int t = threadIdx.x;
    s0[t] = lo;
    s1[t] = hi;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (t < h) {
            s0[t] = fmin(s0[t], s0[t + h]);
            double a = s1[t], b = s1[t + h];
            s1[t] = (a != a || b != b) ? NAN : fmax(a, b);
        }
        __syncthreads();
    }
    if (t == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// Copy the reported potentials out, gauge-fixed so that sum(u) = sum(v) (the dual is
// invariant under (u + delta, v - delta), paper Sec. 4.1 footnote).
__global__ void k_finish(const Work* __restrict__ wp, double* u_out, double* v_out)
{
    const Work w = *wp;
    __shared__ double sred[kWG];
    __shared__ double sdelta;
    const int n = w.n, t = threadIdx.x;
    const double* zb = w.zbest;
    double s = 0.0;
    for (int i = t; i < n; i += kWG) s += zb[n + i] - zb[i];
    sred[t] = s;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (t < h) sred[t] += sred[t + h];
        __syncthreads();
    }
    if (t == 0) sdelta = sred[0] / (2.0 * n);
    __syncthreads();
    const double dl = sdelta;
    for (int i = t; i < n; i += kWG) {
        if (u_out) u_out[i] = zb[i] + dl;
        if (v_out) v_out[i] = zb[n + i] - dl;
    }
}

// ------------------------------------------------------------------ launchers
int launch_step(const Work* wd, int n, int tiles, int parity, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_ctrl, dim3((2 * n + kVecWG - 1) / kVecWG), dim3(kVecWG), 0, s, wd, parity);
    hipLaunchKernelGGL(k_sweep, dim3(tiles), dim3(kWG), 0, s, wd, parity);
    hipLaunchKernelGGL(k_round, dim3(tiles), dim3(kWG), 0, s, wd, parity);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_init(const Work* wd, void* stream)
{
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, (hipStream_t)stream, wd);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_intake(const Work* wd, double* out8, void* stream)
{
    hipLaunchKernelGGL(k_intake, dim3(1), dim3(kWG), 0, (hipStream_t)stream, wd, out8);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cost_range(const Work* wd, int tiles, double* part, void* stream)
{
    hipLaunchKernelGGL(k_cost_range, dim3(tiles), dim3(kWG), 0, (hipStream_t)stream, wd, part);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_finish(const Work* wd, double* u_out, double* v_out, void* stream)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, (hipStream_t)stream, wd, u_out, v_out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mdot
