// Dense-state kernels (16 < m <= 32; built for the 20 amino-acid states) with
// FP64 or FP32 partial vectors.  Every product of a transition matrix, its
// transpose, Q or Q^2 with a partial vector is a (16-row block) x 16-pattern
// product on the matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32,
// accumulation in the vectors' type).  The passes compute what the
// small-state kernels compute (Sections 2.3-2.7): post-order messages
// m_k = P_k p~_k, per-category root values and scale exponents, pre-order
// vectors q, the per-branch ratio (u^T Q m) / (u^T m) weighted by
// w_s rho_{s,l} gamma_l, and for the Hessian (u^T Q^2 m) / (u^T m).
//
// Register and memory layout (see the dense-state notes in pg_internal.h).
// A wave owns one tile (16 consecutive patterns of one category) of one node
// at a time; lane L = 16 g + c holds pattern c, row block 0 (the states
// dn_b0_state(g, r), r < 4: 4 g + r in FP32, g + 4 r in FP64, the matrix
// cores' accumulator order) as one 4-vector and the K1 states 16 + K1 g + r
// of row block 1.  In HBM one tile of a vector is [block 0: 64 lanes x 4][block 1:
// 64 lanes x K1] (M = 20: 2 KB + 512 B in FP64, whole-wave runs).
//
// Transition-matrix slots, per (branch, category), in the vectors' type: an
// internal branch holds the A fragments of P (post-order P p) and of P^T
// (pre-order P^T u); a tip branch holds the table of P's columns (row y < m:
// column y, the message of an observed state y; row m: P 1, the message of
// missing data).  Q and Q^2 fragments come from the host.
//
// Work decomposition as the split-BF16 kernels: a workgroup of waves owns
// one tile and walks the tree level by level (nodes of one height are
// independent; a barrier separates levels), one node per wave at a time;
// the post-order pass issues the next node's loads before the current
// node's arithmetic, the pre-order pass (more registers per wave) does not.
// Tiles are mapped to workgroups XCD by XCD.
#include <type_traits>

#include "device_common.h"
#include "expm_lds.h"

namespace pg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T>
using v4 = typename std::conditional<sizeof(T) == 8, d4, f4>::type;

__device__ inline d4 mma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// waves per traversal workgroup: the post-order kernel runs more, smaller
// workgroups (its FP64 variant holds fewer registers and keeps three
// workgroups of four waves per CU); the pre-order kernel eight
constexpr int DW_POST = 4, DW_PRE = 8;

// The lane's M states of its pattern: row block 0 and the K1 rows of block 1.
template <int M, typename T>
struct DV {
    v4<T> b0;
    T b1[dn_k1(M)];
};

template <int M, typename T>
__device__ inline void dzero(DV<M, T>& v) {
    v.b0 = v4<T>{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int r = 0; r < dn_k1(M); ++r) v.b1[r] = T(0);
}

template <int M, typename T>
__device__ inline DV<M, T> dmul(const DV<M, T>& a, const DV<M, T>& b) {
    DV<M, T> o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o.b0[i] = a.b0[i] * b.b0[i];
#pragma unroll
    for (int r = 0; r < dn_k1(M); ++r) o.b1[r] = a.b1[r] * b.b1[r];
    return o;
}

// the lane's part of a^T b (padding entries are zero)
template <int M, typename T>
__device__ inline T ddot(const DV<M, T>& a, const DV<M, T>& b) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) s = fma(a.b0[i], b.b0[i], s);
#pragma unroll
    for (int r = 0; r < dn_k1(M); ++r) s = fma(a.b1[r], b.b1[r], s);
    return s;
}

// reductions over the four lane groups holding the same pattern; every
// lane gets the same bits
template <typename T>
__device__ inline T dsum4(T v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
}
template <typename T>
__device__ inline T dmax4(T v) {
    v = fmax(v, __shfl_xor(v, 16));
    return fmax(v, __shfl_xor(v, 32));
}

template <int M>
__device__ inline size_t dvec_off(const EvalArgs& a, int node, int tile) {
    return ((size_t)(node - a.n_tips) * a.n_tiles + tile) * (size_t)(dn_md(M) * TP);
}

template <int M, typename T>
__device__ inline void dload(const T* base, int lane, DV<M, T>& v) {
    constexpr int K1 = dn_k1(M);
    v.b0 = reinterpret_cast<const v4<T>*>(base)[lane];
#pragma unroll
    for (int r = 0; r < K1; ++r) v.b1[r] = base[256 + lane * K1 + r];
}

template <int M, typename T>
__device__ inline void dstore(T* base, int lane, const DV<M, T>& v) {
    constexpr int K1 = dn_k1(M);
    reinterpret_cast<v4<T>*>(base)[lane] = v.b0;
#pragma unroll
    for (int r = 0; r < K1; ++r) base[256 + lane * K1 + r] = v.b1[r];
}

template <int M, typename T>
__device__ inline const T* dslot(const EvalArgs& a, int b, int l) {
    return static_cast<const T*>(a.P) + ((size_t)b * a.K + l) * dn_slot_elems(M);
}

// A fragments of one matrix ([ob][s][lane]), issued together
template <int M, typename T>
__device__ inline void frags_load(const T* __restrict__ src, int lane, T f[dn_nf(M)]) {
#pragma unroll
    for (int i = 0; i < dn_nf(M); ++i) f[i] = src[i * 64 + lane];
}

// y = A x with A's fragments f[ob * KS + s]; the two output row blocks
// alternate so consecutive MFMAs are independent
template <int M, typename T>
__device__ inline void dprod(const T f[dn_nf(M)], const DV<M, T>& x, DV<M, T>& y) {
    constexpr int KS = dn_ks(M), K1 = dn_k1(M);
    v4<T> a0 = {T(0), T(0), T(0), T(0)}, a1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        a0 = mma(f[s], x.b0[s], a0);
        a1 = mma(f[KS + s], x.b0[s], a1);
    }
#pragma unroll
    for (int s = 0; s < K1; ++s) {
        a0 = mma(f[4 + s], x.b1[s], a0);
        a1 = mma(f[KS + 4 + s], x.b1[s], a1);
    }
    y.b0 = a0;
#pragma unroll
    for (int r = 0; r < K1; ++r) y.b1[r] = a1[r];
}

// Scale v by 2^-e, e the exponent of its largest entry over the pattern's
// states; returns e (0 for an all-zero vector).
template <int M, typename T>
__device__ inline int drescale(DV<M, T>& v) {
    T mx = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) mx = fmax(mx, v.b0[i]);
#pragma unroll
    for (int r = 0; r < dn_k1(M); ++r) mx = fmax(mx, v.b1[r]);
    mx = dmax4(mx);
    if (!(mx > T(0))) return 0;
    const int e = exp_of(mx);
#pragma unroll
    for (int i = 0; i < 4; ++i) v.b0[i] = pow2_scale(v.b0[i], -e);
#pragma unroll
    for (int r = 0; r < dn_k1(M); ++r) v.b1[r] = pow2_scale(v.b1[r], -e);
    return e;
}

// the root distribution pi in the lane's layout
template <int M, typename T>
__device__ inline void droot_q(const EvalArgs& a, int lane, DV<M, T>& q) {
    constexpr int K1 = dn_k1(M);
    const int g = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) q.b0[i] = T(a.pi64[dn_b0_state(g, i, sizeof(T) == 8)]);
#pragma unroll
    for (int r = 0; r < K1; ++r) {
        const int x = 16 + K1 * g + r;
        q.b1[r] = x < M ? T(a.pi64[x]) : T(0);
    }
}

// ---------------------------------------------------------------- children
//
// Outgoing message of child c (Section 2.1): the stored m_c of an internal
// child; for a tip, P_c times the tip indicator: one row of the tip table
// (observed state, or the all-ones row), or the sum of the allowed rows.
template <int M, typename T>
struct DChild {
    DV<M, T> v;
    unsigned code;
};

template <int M, typename T>
__device__ inline void dchild_issue(const EvalArgs& a, int c, int tile, int s, int lane, DChild<M, T>& r) {
    if (c >= a.n_tips) dload(static_cast<const T*>(a.msg) + dvec_off<M>(a, c, tile), lane, r.v);
    else r.code = a.codes[(size_t)c * a.S_pad + s];
}

template <int M, typename T>
__device__ inline void dchild_finish(const EvalArgs& a, int c, int l, int lane, const DChild<M, T>& r,
                                     DV<M, T>& out) {
    constexpr int K1 = dn_k1(M), MD = dn_md(M);
    if (c >= a.n_tips) {
        out = r.v;
        return;
    }
    const int g = lane >> 4;
    const T* tab = dslot<M, T>(a, c, l);
    const unsigned code = r.code;
    const int row = code < (unsigned)M ? (int)code : (code == 255u ? M : -1);
    if (row >= 0) {
        const T* src = tab + row * MD;
        out.b0 = *reinterpret_cast<const v4<T>*>(src + 4 * g);
#pragma unroll
        for (int k = 0; k < K1; ++k) out.b1[k] = src[16 + K1 * g + k];
    } else {
        const unsigned long long mask = a.masks[code];
        dzero(out);
        for (int y = 0; y < M; ++y)
            if ((mask >> y) & 1ull) {
                const T* src = tab + y * MD;
                const v4<T> b0 = *reinterpret_cast<const v4<T>*>(src + 4 * g);
#pragma unroll
                for (int i = 0; i < 4; ++i) out.b0[i] += b0[i];
#pragma unroll
                for (int k = 0; k < K1; ++k) out.b1[k] += src[16 + K1 * g + k];
            }
    }
}

// ---------------------------------------------------------------- transition matrices

template <int M, typename T>
__device__ inline void dense_pmat_body(const EvalArgs& a, int block) {
    constexpr int NF = dn_nf(M), KS = dn_ks(M), MD = dn_md(M);
    constexpr bool wide = sizeof(T) == 8;
    __shared__ double A[M * M], G[M * M], W[M * M], fc[M], fs[M];
    const int b = a.blist ? a.blist[block / a.K] : block / a.K, l = block % a.K;
    T* slot = static_cast<T*>(a.P) + ((size_t)b * a.K + l) * dn_slot_elems(M);
    // eigen route when the host found Q usably diagonalisable (homogeneous
    // model), scaling and squaring otherwise
    const bool ok = (!a.expm_taylor && a.n_models == 0) ? eigen_F_lds<M>(a, b, l, A, G, W, fc, fs)
                                                         : taylor_F_lds<M>(a, b, l, A, G, W);
    // W = F, P = I + F
    auto pent = [&](int x, int y) { return ((x == y) ? 1.0 : 0.0) + W[x * M + y]; };
    if (b >= a.n_tips) {
        // fragments [which][ob][s][lane]: which 0 = P, 1 = P^T
        for (int e = threadIdx.x; e < 2 * NF * 64; e += blockDim.x) {
            const int which = e / (NF * 64), f = (e / 64) % NF, L = e % 64;
            const int x = dn_row_state(M, f / KS, L % 16, wide), y = dn_col_state(M, f % KS, L / 16, wide);
            double v = 0.0;
            if (ok && x >= 0 && y >= 0) v = which == 0 ? pent(x, y) : pent(y, x);
            slot[e] = ok ? T(v) : T(NAN);
        }
    } else {
        // tip table: row y < M = column y of P, row M = P 1 (1 + row sums of
        // F), entries in the lanes' register order
        for (int e = threadIdx.x; e < (M + 1) * MD; e += blockDim.x) {
            const int y = e / MD, j = e % MD;
            const int x = j < 16 ? dn_b0_state(j / 4, j % 4, wide) : j;
            double v = 0.0;
            if (ok && x < M) {
                if (y < M) {
                    v = pent(x, y);
                } else {
                    double sum = 0.0;
                    for (int z = 0; z < M; ++z) sum += W[x * M + z];
                    v = 1.0 + sum;
                }
            }
            slot[e] = ok ? T(v) : T(NAN);
        }
    }
}

// ---------------------------------------------------------------- post-order pass
//
// For each internal node k (children i, j), category l, pattern s:
//   p_k = m_i o m_j, rescaled        Eq. (postOrderPartialUpdate)
//   m_k = P_k p~_k stored unless k is the root; at the root pi^T p~_root
//   (Eq. rootInnerProduct) and the pattern's summed exponents.

template <int M, typename T>
__device__ inline void dense_post_node(const EvalArgs& a, int4 nd, int l, int tile, int s, int lane,
                                       const DChild<M, T>& ci, const DChild<M, T>& cj, int& esum) {
    constexpr int NF = dn_nf(M), K1 = dn_k1(M);
    const int g = lane >> 4, ps = lane & 15;
    const bool has_msg = nd.x != a.root;
    T f[NF];
    if (has_msg) frags_load<M, T>(dslot<M, T>(a, nd.x, l), lane, f);
    DV<M, T> mi, mj;
    dchild_finish<M, T>(a, nd.y, l, lane, ci, mi);
    dchild_finish<M, T>(a, nd.z, l, lane, cj, mj);
    DV<M, T> p = dmul(mi, mj);
    const int e = drescale(p);
    if (a.expo) {
        // per-node exponents for partial re-evaluation (lane group 0 owns
        // them): a pass over some nodes adds the change of each visited
        // node's exponent
        if (g == 0) {
            int16_t* ex = a.expo + ((size_t)(nd.x - a.n_tips) * a.n_tiles + tile) * TP + ps;
            esum += a.expo_delta ? e - (int)*ex : e;
            *ex = (int16_t)e;
        }
    } else {
        esum += e;
    }
    if (has_msg) {
        DV<M, T> m;
        dprod<M, T>(f, p, m);
        dstore<M, T>(static_cast<T*>(a.msg) + dvec_off<M>(a, nd.x, tile), lane, m);
    } else {
        double Lt = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) Lt = fma(a.pi64[dn_b0_state(g, i, sizeof(T) == 8)], (double)p.b0[i], Lt);
#pragma unroll
        for (int r = 0; r < K1; ++r) {
            const int x = 16 + K1 * g + r;
            if (x < M) Lt = fma(a.pi64[x], (double)p.b1[r], Lt);
        }
        Lt = dsum4(Lt);
        if (g == 0) a.rootL[(size_t)l * a.S_pad + s] = Lt;
    }
}

template <int M, typename T>
__device__ inline void dense_post_body(const EvalArgs& a, int tile, int4* lds_sched) {
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ps = lane & 15, g = lane >> 4;
    const int s = pb * TP + ps;
    stage_schedule(a, lds_sched);
    int esum = 0;
    for (int h = 0; h < a.n_levels; ++h) {
        const int end = a.level_off[h + 1];
        int idx = a.level_off[h] + wv;
        if (idx < end) {
            // software pipeline: the next node's loads go out before this
            // node's arithmetic and stores
            int4 nd = sched_at(a, lds_sched, idx);
            DChild<M, T> ci, cj;
            dchild_issue<M, T>(a, nd.y, tile, s, lane, ci);
            dchild_issue<M, T>(a, nd.z, tile, s, lane, cj);
            while (true) {
                const int nidx = idx + DW_POST;
                const bool more = nidx < end;
                int4 nn = nd;
                DChild<M, T> ni, nj;
                if (more) {
                    nn = sched_at(a, lds_sched, nidx);
                    dchild_issue<M, T>(a, nn.y, tile, s, lane, ni);
                    dchild_issue<M, T>(a, nn.z, tile, s, lane, nj);
                }
                dense_post_node<M, T>(a, nd, l, tile, s, lane, ci, cj, esum);
                if (!more) break;
                nd = nn;
                ci = ni;
                cj = nj;
                idx = nidx;
            }
        }
        __syncthreads();
    }
    __shared__ int red[DW_POST][TP];
    if (g == 0) red[wv][ps] = esum;
    __syncthreads();
    if (wv == 0 && g == 0) {
        int tot = 0;
        for (int i = 0; i < DW_POST; ++i) tot += red[i][ps];
        if (a.expo_delta) a.rootE[(size_t)l * a.S_pad + s] += tot;
        else a.rootE[(size_t)l * a.S_pad + s] = tot;
    }
}

// ---------------------------------------------------------------- pre-order pass + gradient
//
// For each internal node k (q_root = pi), category l, pattern s, and each
// child c with sibling b:
//   u = q~_k o m_b, ratio = (u^T Q m_c) / (u^T m_c)     Eq. (singleRateCaseGradient)
//   tile sum of w_s rho_{s,l} gamma_l ratio               Eq. (GradientWithGamma)
//   q_c = P_c^T u, rescaled, stored if c is internal      Eq. (preOrderUpdate)
// HESS adds the tile sums of w_s rho gamma^2 (u^T Q^2 m)/(u^T m) and the
// per-pattern rho gamma ratio (Section 2.7, reduced by hsum_kernel).

template <int M, typename T, bool HESS, bool NH>
__device__ inline void dense_pre_child(const EvalArgs& a, int c, int l, int tile, int s, int lane, const Coef& cf,
                                       const DV<M, T>& u, const DV<M, T>& mown, const T* qf,
                                       const T* q2f, const T pf[dn_nf(M)]) {
    constexpr int NF = dn_nf(M);
    const int g = lane >> 4;
    T den = ddot(u, mown);
    DV<M, T> qm;
    T num, num2 = T(0);
    if constexpr (NH) {
        // Q and Q^2 of branch c's rate matrix
        const T* QF = static_cast<const T*>(a.Qfrag) + (size_t)a.branch_model[c] * dn_qfrag_elems(M);
        T f[NF];
        frags_load<M, T>(QF, lane, f);
        dprod<M, T>(f, mown, qm);
        num = ddot(u, qm);
        if constexpr (HESS) {
            frags_load<M, T>(QF + NF * 64, lane, f);
            DV<M, T> q2m;
            dprod<M, T>(f, mown, q2m);
            num2 = ddot(u, q2m);
        }
    } else {
        T f[NF];
        frags_load<M, T>(qf, lane, f);
        dprod<M, T>(f, mown, qm);
        num = ddot(u, qm);
        if constexpr (HESS) {
            frags_load<M, T>(q2f, lane, f);
            DV<M, T> q2m;
            dprod<M, T>(f, mown, q2m);
            num2 = ddot(u, q2m);
        }
    }
    den = dsum4(den);
    num = dsum4(num);
    const double ratio = (den > T(0)) ? (double)num / (double)den : 0.0;
    double term = (cf.g > 0.0) ? cf.g * ratio : 0.0;
    term = sum16(term);  // every row holds the same 16 patterns
    if (lane == 0) a.partial[(size_t)tile * a.n_branches + c] = term;
    if constexpr (HESS) {
        num2 = dsum4(num2);
        const double ratio2 = (den > T(0)) ? (double)num2 / (double)den : 0.0;
        double term2 = (cf.h > 0.0) ? cf.h * ratio2 : 0.0;
        term2 = sum16(term2);
        if (lane == 0) a.partial2[(size_t)tile * a.n_branches + c] = term2;
        if (g == 0) a.r1[((size_t)c * a.K + l) * a.S_pad + s] = (cf.nw > 0.0) ? cf.nw * ratio : 0.0;
    }
    if (c >= a.n_tips) {
        DV<M, T> qc;
        dprod<M, T>(pf, u, qc);
        (void)drescale(qc);
        dstore<M, T>(static_cast<T*>(a.qv) + dvec_off<M>(a, c, tile), lane, qc);
    }
}

// loads of one pre-order node: its q (not the root's) and the children's
// messages (internal) or tip codes
template <int M, typename T>
struct DPreLd {
    DV<M, T> q;
    DChild<M, T> ci, cj;
};

template <int M, typename T>
__device__ inline void dpre_issue(const EvalArgs& a, int4 nd, int tile, int s, int lane, DPreLd<M, T>& r) {
    if (nd.x != a.root) dload(static_cast<const T*>(a.qv) + dvec_off<M>(a, nd.x, tile), lane, r.q);
    dchild_issue<M, T>(a, nd.y, tile, s, lane, r.ci);
    dchild_issue<M, T>(a, nd.z, tile, s, lane, r.cj);
}

template <int M, typename T, bool HESS, bool NH>
__device__ inline void dense_pre_body(const EvalArgs& a, int tile, int4* lds_sched) {
    constexpr int NF = dn_nf(M);
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ps = lane & 15, g = lane >> 4;
    const int s = pb * TP + ps;
    // rho_{s,l} gamma_l w_s from the per-category root values
    Coef cf;
    {
        const SiteLik r = site_likelihood(a, s);
        cf = coef_of(a, l, s, r);
        // the category-0 tile of each pattern block also forms its logL part
        if (l == 0 && wv == 0 && g == 0) logl_block_part(a, pb, ps, r);
    }
    // Q (and Q^2) fragments of the homogeneous model are staged in LDS; each
    // product reloads them (in registers they would cost a wave per SIMD)
    __shared__ T qsh[2 * NF * 64];
    if constexpr (!NH) {
        const T* QF = static_cast<const T*>(a.Qfrag);
        for (int i = threadIdx.x; i < (HESS ? 2 : 1) * NF * 64; i += blockDim.x) qsh[i] = QF[i];
        __syncthreads();
    }
    const T* qf = qsh;
    const T* q2f = qsh + NF * 64;
    stage_schedule(a, lds_sched);
    for (int h = a.n_levels - 1; h >= 0; --h) {
        const int end = a.level_off[h + 1];
        int idx = a.level_off[h] + wv;
        if (idx < end) {
            int4 nd = sched_at(a, lds_sched, idx);
            DPreLd<M, T> cur;
            dpre_issue<M, T>(a, nd, tile, s, lane, cur);
            while (true) {
                const int nidx = idx + DW_PRE;
                const bool more = nidx < end;
                int4 nn = nd;
                if (more) nn = sched_at(a, lds_sched, nidx);
                T pf[NF];
                if (nd.y >= a.n_tips) frags_load<M, T>(dslot<M, T>(a, nd.y, l) + NF * 64, lane, pf);
                DV<M, T> q;
                if (nd.x == a.root) droot_q<M, T>(a, lane, q);
                else q = cur.q;
                DV<M, T> mi, mj;
                dchild_finish<M, T>(a, nd.y, l, lane, cur.ci, mi);
                dchild_finish<M, T>(a, nd.z, l, lane, cur.cj, mj);
                const DV<M, T> ui = dmul(q, mj), uj = dmul(q, mi);
                dense_pre_child<M, T, HESS, NH>(a, nd.y, l, tile, s, lane, cf, ui, mi, qf, q2f, pf);
                if (nd.z >= a.n_tips) frags_load<M, T>(dslot<M, T>(a, nd.z, l) + NF * 64, lane, pf);
                dense_pre_child<M, T, HESS, NH>(a, nd.z, l, tile, s, lane, cf, uj, mj, qf, q2f, pf);
                if (!more) break;
                nd = nn;
                dpre_issue<M, T>(a, nd, tile, s, lane, cur);
                idx = nidx;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- entry points
//
// Single-evaluation kernels map block b to tile xcd_tile(b); the batched
// kernels of the serving scheduler take {request, block} from map[].

template <int M, typename T>
__global__ void __launch_bounds__(256) dense_pmat_kernel(EvalArgs a) { dense_pmat_body<M, T>(a, blockIdx.x); }
template <int M, typename T>
__global__ void __launch_bounds__(256) dense_pmat_batch(const EvalArgs* __restrict__ reqs,
                                                         const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    dense_pmat_body<M, T>(reqs[m.x], m.y);
}

template <int M, typename T>
__global__ void __launch_bounds__(DW_POST * 64) dense_post_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    dense_post_body<M, T>(a, tile, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(DW_POST * 64) dense_post_batch(const EvalArgs* __restrict__ reqs,
                                                                const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    dense_post_body<M, T>(reqs[m.x], m.y, lds_dyn);
}

template <int M, typename T, bool HESS, bool NH>
__global__ void __launch_bounds__(DW_PRE * 64) dense_pre_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    dense_pre_body<M, T, HESS, NH>(a, tile, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(DW_PRE * 64) dense_pre_batch(const EvalArgs* __restrict__ reqs,
                                                               const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    dense_pre_body<M, T, false, false>(reqs[m.x], m.y, lds_dyn);
}

// ---------------------------------------------------------------- dispatch (M = 20)

template <int M, typename T>
static hipError_t dpmat(const EvalArgs& a, hipStream_t st) {
    dense_pmat_kernel<M, T><<<(a.blist ? a.n_blist : a.n_branches) * a.K, 256, 0, st>>>(a);
    return hipGetLastError();
}
template <int M, typename T>
static hipError_t dpost(const EvalArgs& a, hipStream_t st) {
    dense_post_kernel<M, T><<<N_XCD * xcd_per(a.n_tiles), DW_POST * 64, sched_lds_bytes(a), st>>>(a);
    return hipGetLastError();
}
template <int M, typename T>
static hipError_t dpre(const EvalArgs& a, hipStream_t st, bool hess) {
    const dim3 grid(N_XCD * xcd_per(a.n_tiles)), block(DW_PRE * 64);
    const size_t lds = sched_lds_bytes(a);
    if (a.n_models) {
        if (hess) dense_pre_kernel<M, T, true, true><<<grid, block, lds, st>>>(a);
        else dense_pre_kernel<M, T, false, true><<<grid, block, lds, st>>>(a);
    } else {
        if (hess) dense_pre_kernel<M, T, true, false><<<grid, block, lds, st>>>(a);
        else dense_pre_kernel<M, T, false, false><<<grid, block, lds, st>>>(a);
    }
    return hipGetLastError();
}
template <int M, typename T>
static hipError_t dbatch(const BatchLaunch& b, hipStream_t st) {
    if (b.pmat_blocks > 0) dense_pmat_batch<M, T><<<b.pmat_blocks, 256, 0, st>>>(b.reqs, b.pmat_map);
    dense_post_batch<M, T><<<b.trav_blocks, DW_POST * 64, b.post_lds, st>>>(b.reqs, b.trav_map);
    dense_pre_batch<M, T><<<b.trav_blocks, DW_PRE * 64, b.pre_lds, st>>>(b.reqs, b.trav_map);
    return hipGetLastError();
}

hipError_t launch_dense_pmat(const EvalArgs& a, int precision, hipStream_t st) {
    if (a.M == 20 && precision == PG_FP64) return dpmat<20, double>(a, st);
    if (a.M == 20 && precision == PG_FP32) return dpmat<20, float>(a, st);
    return hipErrorInvalidValue;
}
hipError_t launch_dense_post(const EvalArgs& a, int precision, hipStream_t st) {
    if (a.M == 20 && precision == PG_FP64) return dpost<20, double>(a, st);
    if (a.M == 20 && precision == PG_FP32) return dpost<20, float>(a, st);
    return hipErrorInvalidValue;
}
hipError_t launch_dense_pre(const EvalArgs& a, int precision, hipStream_t st, bool hess) {
    if (a.M == 20 && precision == PG_FP64) return dpre<20, double>(a, st, hess);
    if (a.M == 20 && precision == PG_FP32) return dpre<20, float>(a, st, hess);
    return hipErrorInvalidValue;
}
// pmat, post and pre of a serving batch (the caller launches the reduction)
hipError_t launch_dense_batch(const BatchLaunch& b, hipStream_t st) {
    if (b.M == 20 && b.precision == PG_FP64) return dbatch<20, double>(b, st);
    if (b.M == 20 && b.precision == PG_FP32) return dbatch<20, float>(b, st);
    return hipErrorInvalidValue;
}

}  // namespace pg
