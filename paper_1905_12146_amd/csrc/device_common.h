// Device helpers shared by the kernels of every precision: exact power-of-
// two rescaling, DPP row reductions, tip codes, the level schedule, and the
// per-site likelihood from the per-category root values.
#pragma once

#include <climits>

#include "pg_internal.h"

namespace pg {

// XCD-aware tile order: workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8), so block b takes tile
// (b % 8) * per + b / 8 and each XCD walks a contiguous range of tiles: one
// or two categories, whose transition-matrix fragments then stay in that
// XCD's L2 while its tiles walk the same tree levels.  The grid has
// 8 * per blocks; blocks past the last tile return at once.
constexpr int N_XCD = 8;
__host__ __device__ inline int xcd_per(int n_tiles) { return (n_tiles + N_XCD - 1) / N_XCD; }
__device__ inline int xcd_tile(int b, int n_tiles) { return (b % N_XCD) * xcd_per(n_tiles) + b / N_XCD; }


__device__ inline int exp_of(double x) { int e; (void)frexp(x, &e); return e; }
__device__ inline int exp_of(float x) { int e; (void)frexpf(x, &e); return e; }
__device__ inline double pow2_scale(double x, int e) { return ldexp(x, e); }
__device__ inline float pow2_scale(float x, int e) { return ldexpf(x, e); }

// Sum over the 16 lanes of a node slot (one DPP row).  Each step adds the
// row rotated by 1, 2, 4, 8 lanes (v_mov_b32_dpp row_ror on both halves of
// the double), so every lane ends with the full row sum; callers use lane 0's
// value, whose association order is fixed.
template <int N>
__device__ inline double row_ror(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x120 + N, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x120 + N, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ inline double sum16(double v) {
    v += row_ror<1>(v);
    v += row_ror<2>(v);
    v += row_ror<4>(v);
    v += row_ror<8>(v);
    return v;
}

// Any 32-bit DPP control on both halves of a double.
template <int CTRL>
__device__ inline double dpp64(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// The row sums of a and of b together (upper: lane 8-15 of its row): the
// first step leaves a_i + a_{i+8} in lanes 0-7 and b_i + b_{i-8} in lanes
// 8-15 (each lane sends its partner half the value that half sums), then
// each half of the row is summed by a mirror and two quad exchanges.  Lane
// 0 of the row ends with the sum of a, lane 8 with the sum of b, each in a
// fixed association order.
__device__ inline double pair_sum16(double a, double b, bool upper) {
    double v = (upper ? b : a) + row_ror<8>(upper ? a : b);
    v += dpp64<0x141>(v);  // row_half_mirror
    v += dpp64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    return v;
}

__device__ inline unsigned long long tip_mask(const EvalArgs& a, unsigned code, int M) {
    if (code < (unsigned)M) return 1ull << code;
    if (code == 255u) return ~0ull;
    return a.masks[code];
}

// Level-ordered schedule entry idx: {node, child 0, child 1, 0}, from LDS
// when the schedule was staged there.
// An LDS read through an LDS-typed pointer: a select between the staged
// copy and global memory would otherwise become one generic (flat) load,
// whose wait also drains every outstanding global load.
typedef __attribute__((address_space(3))) const int lds_int;
__device__ inline int4 lds_entry(const int4* lds, int idx) {
    const lds_int* p = (const lds_int*)(lds + idx);
    return make_int4(p[0], p[1], p[2], p[3]);
}

__device__ inline int4 sched_at(const EvalArgs& a, const int4* lds, int idx) {
    if (a.sched_lds) return lds_entry(lds, idx);
    return a.sched[idx];
}

// Stages the level schedule in LDS.
__device__ inline void stage_schedule(const EvalArgs& a, int4* lds) {
    if (a.sched_lds) {
        for (int i = threadIdx.x; i < a.n_sched; i += blockDim.x) lds[i] = a.sched[i];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- per-site likelihood
//
// L_s = sum_l w_l L~_{s,l} 2^{E_{s,l}}  (Eq. discreteRateLikelihood), formed
// relative to the largest exponent so nothing under- or overflows.

struct SiteLik {
    double scaled;  // L_s 2^-emax
    int emax;
    bool nan;
};

// The categories are read SL_CHUNK at a time, every load of a chunk issued
// before any is used (one memory round trip per chunk, not per category);
// the sums still run over l in increasing order.
constexpr int SL_CHUNK = 4;

__device__ inline SiteLik site_likelihood(const EvalArgs& a, int s) {
    SiteLik r{0.0, INT_MIN, false};
    for (int l0 = 0; l0 < a.K; l0 += SL_CHUNK) {
        double L[SL_CHUNK];
        int E[SL_CHUNK];
#pragma unroll
        for (int c = 0; c < SL_CHUNK; ++c) {
            const size_t at = (size_t)min(l0 + c, a.K - 1) * a.S_pad + s;
            L[c] = a.rootL[at];
            E[c] = a.rootE[at];
        }
#pragma unroll
        for (int c = 0; c < SL_CHUNK; ++c) {
            if (l0 + c < a.K) {
                if (isnan(L[c])) r.nan = true;
                if (L[c] > 0.0) r.emax = max(r.emax, E[c]);
            }
        }
    }
    if (r.emax != INT_MIN)
        for (int l0 = 0; l0 < a.K; l0 += SL_CHUNK) {
            double L[SL_CHUNK];
            int E[SL_CHUNK];
#pragma unroll
            for (int c = 0; c < SL_CHUNK; ++c) {
                const size_t at = (size_t)min(l0 + c, a.K - 1) * a.S_pad + s;
                L[c] = a.rootL[at];
                E[c] = a.rootE[at];
            }
#pragma unroll
            for (int c = 0; c < SL_CHUNK; ++c) {
                if (l0 + c < a.K && L[c] > 0.0) r.scaled += a.catw[l0 + c] * ldexp(L[c], E[c] - r.emax);
            }
        }
    return r;
}

// logL = sum_s w_s log L_s in one fixed order, shared by every path:
//   part[pb] = butterfly sum over the TP patterns of block pb (sum16),
//   logL     = fixed reduction of part[0..n_pb) (finish_logl).
// site_log_term gives one pattern's term and status flag.
__device__ inline double site_log_term(const EvalArgs& a, int s, const SiteLik& r, int& flag) {
    const double LN2 = 0.69314718055994530942;
    const double w = a.weights[s];
    flag = 0;
    if (r.nan) { flag = 1; return 0.0; }
    if (r.scaled > 0.0) return (w > 0.0) ? w * (log(r.scaled) + (double)r.emax * LN2) : 0.0;
    if (w > 0.0) flag = 2;
    return 0.0;
}

__device__ inline int or16(int v) {
    v |= __builtin_amdgcn_mov_dpp(v, 0x121, 0xf, 0xf, false);
    v |= __builtin_amdgcn_mov_dpp(v, 0x122, 0xf, 0xf, false);
    v |= __builtin_amdgcn_mov_dpp(v, 0x124, 0xf, 0xf, false);
    v |= __builtin_amdgcn_mov_dpp(v, 0x128, 0xf, 0xf, false);
    return v;
}

// One 16-lane row computes part[pb] (all lanes of the row active).
__device__ inline void logl_block_part(const EvalArgs& a, int pb, int ps, const SiteLik& r) {
    int flag;
    double v = site_log_term(a, pb * TP + ps, r, flag);
    v = sum16(v);
    flag = or16(flag);
    if (ps == 0) {
        a.logl_part[pb] = v;
        a.flag_part[pb] = flag;
    }
}

// Per-lane coefficients of pattern s in category l:
//   g = w_s rho_{s,l} gamma_l      (gradient)
//   nw = rho_{s,l} gamma_l         (per-site gradient part, Hessian)
//   h = w_s rho_{s,l} gamma_l^2    (second-derivative part, Hessian)
// with rho_{s,l} = w_l L_{s,l} / L_s from the root values.
struct Coef {
    double g, nw, h;
};

__device__ inline Coef coef_of(const EvalArgs& a, int l, int s, const SiteLik& r) {
    Coef cf{0.0, 0.0, 0.0};
    const double L = a.rootL[(size_t)l * a.S_pad + s];
    if (!r.nan && r.scaled > 0.0 && L > 0.0) {
        const double rho = a.catw[l] * ldexp(L, a.rootE[(size_t)l * a.S_pad + s] - r.emax) / r.scaled;
        cf.nw = rho * a.rates[l];
        cf.g = a.weights[s] * cf.nw;
        cf.h = cf.g * a.rates[l];
    }
    return cf;
}


// The values site_likelihood and coef_of read for pattern s and category l,
// loaded together so that one memory round trip covers them (the first
// SL_CHUNK categories; site_coef falls back to the two functions above for
// more categories).
struct SiteVals {
    double L[SL_CHUNK], cw[SL_CHUNK];
    int E[SL_CHUNK];
    double Ll, cwl, w, rate;  // category l's root value and weight, w_s, gamma_l
    int El;
};

__device__ inline void site_vals_load(const EvalArgs& a, int l, int s, SiteVals& v) {
#pragma unroll
    for (int c = 0; c < SL_CHUNK; ++c) {
        const int lc = min(c, a.K - 1);
        const size_t at = (size_t)lc * a.S_pad + s;
        v.L[c] = a.rootL[at];
        v.E[c] = a.rootE[at];
        v.cw[c] = a.catw[lc];
    }
    const size_t at = (size_t)l * a.S_pad + s;
    v.Ll = a.rootL[at];
    v.El = a.rootE[at];
    v.cwl = a.catw[l];
    v.w = a.weights[s];
    v.rate = a.rates[l];
}

// site_likelihood and coef_of of category l from the loaded values: the same
// operations in the same order, so the same bits.
__device__ inline Coef site_coef(const EvalArgs& a, int l, int s, const SiteVals& v, SiteLik& r) {
    if (a.K > SL_CHUNK) {
        r = site_likelihood(a, s);
        return coef_of(a, l, s, r);
    }
    r = SiteLik{0.0, INT_MIN, false};
#pragma unroll
    for (int c = 0; c < SL_CHUNK; ++c) {
        if (c < a.K) {
            if (isnan(v.L[c])) r.nan = true;
            if (v.L[c] > 0.0) r.emax = max(r.emax, v.E[c]);
        }
    }
    if (r.emax != INT_MIN)
#pragma unroll
        for (int c = 0; c < SL_CHUNK; ++c) {
            if (c < a.K && v.L[c] > 0.0) r.scaled += v.cw[c] * ldexp(v.L[c], v.E[c] - r.emax);
        }
    Coef cf{0.0, 0.0, 0.0};
    if (!r.nan && r.scaled > 0.0 && v.Ll > 0.0) {
        const double rho = v.cwl * ldexp(v.Ll, v.El - r.emax) / r.scaled;
        cf.nw = rho * v.rate;
        cf.g = v.w * cf.nw;
        cf.h = cf.g * v.rate;
    }
    return cf;
}

}  // namespace pg
