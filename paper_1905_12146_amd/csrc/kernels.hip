// Device kernels of one evaluation: transition matrices, post-order pass,
// pre-order pass fused with the gradient, and the fixed-order reduction of
// per-tile gradient sums together with the logL reduction.
//
// Data layout in HBM:
//   P     [branch][category][x][y]      x = parent state, y = child state
//   msg   [internal node - N][tile][state][TP]   message P_k p~_k
//   qv    [internal node - N][tile][state][TP]   pre-order vector q~_k
//   codes [tip][pattern]                uint8 code of the tip observation
// A tile is TP consecutive patterns of one rate category (tile = l * n_pb +
// pattern block), so one node's data for one tile is a single contiguous run.
//
// Work decomposition: in the level walks a workgroup owns one tile and walks
// its levels (nodes of equal height are independent; a barrier separates
// levels) with NS node slots x TP pattern lanes (post_slots / pre_slots).
// For small M the subtrees below the top (clades) are walked depth first in
// launches of their own, a wavefront per clade list and four tiles, one per
// 16-lane row; the level walk then covers only the nodes above them.  Tiles
// never communicate, so a pass needs no grid-wide synchronisation.
//
// Rescaling is per node, pattern and category, by an exact power of two.
// Categories never mix inside the traversal: the site likelihood
// L_s = sum_l w_l L_{s,l} is formed from each category's scaled root value
// and summed exponent, and the gradient uses
//   d log L_s / dt_b = sum_l rho_{s,l} gamma_l (u^T Q m)/(u^T m),
//   rho_{s,l} = w_l L_{s,l} / L_s,
// which equals Eq. (GradientWithGamma) of Section 2.6: u^T m is L_{s,l} up
// to the category's own scale factor, which cancels in each ratio.
#include "device_common.h"
#include "expm_lds.h"

#include <utility>

namespace pg {

// ---------------------------------------------------------------- helpers

// Entry i of a schedule or clade list, or of the level offsets, with i the
// same across the wavefront: read through the constant address space, so it
// is a scalar load into scalar registers whose wait never holds up the
// vector loads in flight.
typedef const __attribute__((address_space(4))) int* cint_ptr;
__device__ inline int uniform_int(const int* v, int i) { return ((cint_ptr)v)[i]; }
__device__ inline int4 uniform_entry(const int4* list, int i) {
    const cint_ptr p = (cint_ptr)(list + i);
    return make_int4(p[0], p[1], p[2], p[3]);
}

__device__ inline size_t vec_off(const EvalArgs& a, int node, int tile, int M) {
    return ((size_t)(node - a.n_tips) * a.n_tiles + tile) * (size_t)(M * TP);
}

// Small state spaces (M*M <= TP): a node slot is one 16-lane DPP row, and a
// transition matrix is held one entry per lane (lane e holds P[e / M][e % M]),
// loaded with a single coalesced access.  An entry is delivered to every lane
// of the row by a row broadcast (v_mov_b64_dpp row_newbcast), so the matrix
// is never replicated through the vector memory path.
template <int M>
struct RowMat {
    static constexpr bool value = M * M <= TP;
};

// row_newbcast always reads a valid lane, so bound_ctrl only spares the
// compiler from initialising the destination.
template <int E>
__device__ inline double row_bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + E, 0xf, 0xf, true);
}
template <int E>
__device__ inline float row_bcast(float v) {
    return __builtin_amdgcn_update_dpp(0.0f, v, 0x150 + E, 0xf, 0xf, true);
}

template <int M, typename T>
__device__ inline T load_row_entry(const T* __restrict__ mat, int ps) {
    return (ps < M * M) ? mat[ps] : T(0);
}

// All M*M entries of a row-distributed matrix in every lane of the row:
// ent[e] = entry e (row-major).  Each broadcast runs with the whole row active.
template <int M, typename T, int... E>
__device__ inline void row_entries_impl(T pmine, T ent[M * M], std::integer_sequence<int, E...>) {
    ((ent[E] = row_bcast<E>(pmine)), ...);
}
template <int M, typename T>
__device__ inline void row_entries(T pmine, T ent[M * M]) {
    row_entries_impl<M, T>(pmine, ent, std::make_integer_sequence<int, M * M>{});
}

// M = 4: the 16 multiply-adds of a product with a row-distributed 4 x 4
// matrix, each taking its matrix entry straight from the row broadcast
// (v_fmac_f64_dpp / v_fmac_f32_dpp with row_newbcast; the compiler emits a
// separate v_mov_*_dpp per entry instead).  Instruction i adds entry E_i
// times v[i / 4] to out[i % 4]: the accumulators rotate, so each is
// rewritten only every 4th instruction, beyond the 2 wait states a DPP
// instruction needs after a VALU write of any of its operands.  The
// compiler's hazard checks do not look inside inline assembly, so the block
// opens with 5 wait states (DPP after a VALU write of its operands or of
// EXEC) and closes with 2 (for a DPP read of the results right after it).
#define PG_BC(OP, A, X, E) OP " %[a" #A "], %[p], %[x" #X "] row_newbcast:" #E " row_mask:0xf bank_mask:0xf bound_ctrl:1\n"
#define PG_FMAC16(OP, E0, E1, E2, E3, E4, E5, E6, E7, E8, E9, E10, E11, E12, E13, E14, E15)                     \
    "s_nop 4\n" PG_BC(OP, 0, 0, E0) PG_BC(OP, 1, 0, E1) PG_BC(OP, 2, 0, E2) PG_BC(OP, 3, 0, E3)                 \
        PG_BC(OP, 0, 1, E4) PG_BC(OP, 1, 1, E5) PG_BC(OP, 2, 1, E6) PG_BC(OP, 3, 1, E7) PG_BC(OP, 0, 2, E8)    \
            PG_BC(OP, 1, 2, E9) PG_BC(OP, 2, 2, E10) PG_BC(OP, 3, 2, E11) PG_BC(OP, 0, 3, E12)                 \
                PG_BC(OP, 1, 3, E13) PG_BC(OP, 2, 3, E14) PG_BC(OP, 3, 3, E15) "s_nop 1\n"
#define PG_FMAC16_OPERANDS                                                                                    \
    : [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3)                                              \
    : [p] "v"(pmine), [x0] "v"(v[0]), [x1] "v"(v[1]), [x2] "v"(v[2]), [x3] "v"(v[3])

// TRANS: out = P^T v (instruction i uses entry i = 4 x + y: out[y] += P[x][y]
// v[x]); otherwise out = P v (entry 4 (i % 4) + i / 4: out[x] += P[x][y] v[y]).
// Either way each output sums its four terms in increasing order of the
// vector index, as the generic loops below do.
template <typename T, bool TRANS>
__device__ inline void row_fmac44(T pmine, const T v[4], T out[4]) {
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    if constexpr (sizeof(T) == 8) {
        if constexpr (TRANS)
            asm volatile(PG_FMAC16("v_fmac_f64_dpp", 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15)
                         PG_FMAC16_OPERANDS);
        else
            asm volatile(PG_FMAC16("v_fmac_f64_dpp", 0, 4, 8, 12, 1, 5, 9, 13, 2, 6, 10, 14, 3, 7, 11, 15)
                         PG_FMAC16_OPERANDS);
    } else {
        if constexpr (TRANS)
            asm volatile(PG_FMAC16("v_fmac_f32_dpp", 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15)
                         PG_FMAC16_OPERANDS);
        else
            asm volatile(PG_FMAC16("v_fmac_f32_dpp", 0, 4, 8, 12, 1, 5, 9, 13, 2, 6, 10, 14, 3, 7, 11, 15)
                         PG_FMAC16_OPERANDS);
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
}
#undef PG_FMAC16_OPERANDS
#undef PG_FMAC16
#undef PG_BC

// out = P p with P row-distributed (all lanes of the row must be active).
// Entry e = x M + y is broadcast and consumed at once; for each x the sum
// runs over y in increasing order.
template <int M, typename T, int... E>
__device__ inline void row_matvec_impl(T pmine, const T p[M], T out[M], std::integer_sequence<int, E...>) {
#pragma unroll
    for (int x = 0; x < M; ++x) out[x] = T(0);
    ((out[E / M] = fma(row_bcast<E>(pmine), p[E % M], out[E / M])), ...);
}
template <int M, typename T>
__device__ inline void row_matvec(T pmine, const T p[M], T out[M]) {
#ifndef PG_NO_FMAC_DPP
    if constexpr (M == 4) {
        row_fmac44<T, false>(pmine, p, out);
        return;
    }
#endif
    row_matvec_impl<M, T>(pmine, p, out, std::make_integer_sequence<int, M * M>{});
}

// out = P^T u with P row-distributed; for each y the sum runs over x in
// increasing order.
template <int M, typename T, int... E>
__device__ inline void row_matvec_t_impl(T pmine, const T u[M], T out[M], std::integer_sequence<int, E...>) {
#pragma unroll
    for (int y = 0; y < M; ++y) out[y] = T(0);
    ((out[E % M] = fma(row_bcast<E>(pmine), u[E / M], out[E % M])), ...);
}
template <int M, typename T>
__device__ inline void row_matvec_t(T pmine, const T u[M], T out[M]) {
#ifndef PG_NO_FMAC_DPP
    if constexpr (M == 4) {
        row_fmac44<T, true>(pmine, u, out);
        return;
    }
#endif
    row_matvec_t_impl<M, T>(pmine, u, out, std::make_integer_sequence<int, M * M>{});
}

// out[x] = sum_{y in mask} P[x][y] with P row-distributed
template <int M, typename T>
__device__ inline void row_masked_rows(T pmine, unsigned long long mask, T out[M]) {
    T ent[M * M];
    row_entries<M, T>(pmine, ent);
#pragma unroll
    for (int x = 0; x < M; ++x) {
        T acc = T(0);
#pragma unroll
        for (int y = 0; y < M; ++y) acc += ((mask >> y) & 1ull) ? ent[x * M + y] : T(0);
        out[x] = acc;
    }
}

// Q[e] and pi[x]: from the kernel arguments for small M, else from memory
template <int M>
__device__ inline double qentry(const EvalArgs& a, int e) {
    if constexpr (M * M <= 16) return a.Qs[e];
    else return a.Q64[e];
}
template <int M>
__device__ inline double q2entry(const EvalArgs& a, int e) {
    if constexpr (M * M <= 16) return a.Q2s[e];
    else return a.Q2_64[e];
}
template <int M>
__device__ inline double pientry(const EvalArgs& a, int x) {
    if constexpr (M <= 4) return a.pis[x];
    else return a.pi64[x];
}

// Outgoing message of child c for category l, pattern s: the stored
// P_c p~_c of an internal child; for a tip, P_c times the tip indicator
// (Section 2.1): the column of the observed state, or the sum of the allowed
// columns.  Split in two so a node's loads can be issued one node ahead of
// its arithmetic: child_load only issues loads, child_finish uses them.
template <int M, typename T>
struct ChildRaw {
    T v[M];          // internal child: the message; tip (small M): v[0] = own matrix entry
    unsigned code;   // tip code
};

template <int M, typename T>
__device__ inline const T* pmat_of(const EvalArgs& a, int b, int l) {
    return static_cast<const T*>(a.P) + ((size_t)b * a.K + l) * M * M;
}

template <int M, typename T>
__device__ inline void child_load(const EvalArgs& a, int c, int l, int tile, int s, int ps,
                                  ChildRaw<M, T>& r) {
    if (c < a.n_tips) {
        r.code = a.codes[(size_t)c * a.S_pad + s];
        if constexpr (RowMat<M>::value) r.v[0] = load_row_entry<M, T>(pmat_of<M, T>(a, c, l), ps);
    } else {
        const T* src = static_cast<const T*>(a.msg) + vec_off(a, c, tile, M) + ps;
#pragma unroll
        for (int x = 0; x < M; ++x) r.v[x] = src[x * TP];
    }
}

// All lanes of the node slot's row must be active (row broadcasts, shuffles).
template <int M, typename T>
__device__ inline void child_finish(const EvalArgs& a, int c, int l, const ChildRaw<M, T>& r, T out[M]) {
    if (c < a.n_tips) {
        const unsigned code = r.code;
        if constexpr (RowMat<M>::value) {
            // observed state: column `code`, read from the lane holding entry
            // (x, code); ambiguity codes (rare) sum the allowed columns
            const int col = code < (unsigned)M ? (int)code : 0;
#pragma unroll
            for (int x = 0; x < M; ++x) out[x] = __shfl(r.v[0], x * M + col, TP);
            if (__any(code >= (unsigned)M)) {
                T amb[M];
                row_masked_rows<M, T>(r.v[0], tip_mask(a, code, M), amb);
                if (code >= (unsigned)M) {
#pragma unroll
                    for (int x = 0; x < M; ++x) out[x] = amb[x];
                }
            }
        } else {
            const T* Pc = pmat_of<M, T>(a, c, l);
            if (code < (unsigned)M) {
#pragma unroll
                for (int x = 0; x < M; ++x) out[x] = Pc[x * M + code];
            } else {
                const unsigned long long mask = tip_mask(a, code, M);
#pragma unroll
                for (int x = 0; x < M; ++x) {
                    T acc = T(0);
                    for (int y = 0; y < M; ++y)
                        if ((mask >> y) & 1ull) acc += Pc[x * M + y];
                    out[x] = acc;
                }
            }
        }
    } else {
#pragma unroll
        for (int x = 0; x < M; ++x) out[x] = r.v[x];
    }
}

// Top region of the pre-order pass: the levels from a.top_level up to the
// root hold at most one node per node slot; q of their nodes is kept in LDS
// (one M x TP block per region node) and never written to HBM, and the
// levels are separated by LDS-only barriers.  sched.w packs 1-based region
// slots: bits 0-7 the node, 8-15 child 0, 16-23 child 1 (0 = outside).
__device__ inline int rslot(int w, int which) { return (w >> (8 * which)) & 0xff; }

template <typename T>
__device__ inline T* top_buffer(const EvalArgs& a, int4* lds_sched) {
    return reinterpret_cast<T*>(lds_sched + (a.sched_lds ? a.n_sched : 0));
}

template <int M, typename T>
__device__ inline T* top_vec(T* top, int slot, int ps) {
    return top + (size_t)(slot - 1) * (M * TP) + ps;
}

// LDS-only barrier: waits for this wave's LDS operations, not for its
// outstanding global stores.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- transition matrices
//
// P = exp(A), A = Q * rate_l * t_b, by scaling and squaring of the Taylor
// series, carried in the form P = I + F so the small off-diagonal entries
// and the 1 - small diagonal keep full relative accuracy:
//   scale A by 2^-s so that ||A||_inf <= 1/2,
//   F = A (I + A/2 (I + A/3 (... (I + A/DEG)))),      truncation < 1e-19,
//   s times: F <- 2F + F F   ((I+F)^2 = I + 2F + F^2),
//   P = I + F.
// A branch length that is negative or not finite gives a NaN matrix, which
// propagates to a NaN logL.

template <int M>
__device__ inline void matmul_reg(const double A[M][M], const double B[M][M], double C[M][M]) {
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) acc = fma(A[i][k], B[k][j], acc);
            C[i][j] = acc;
        }
}

// One thread per (branch, category); whole matrices in registers (small M).
template <int M, typename T>
__device__ inline void pmat_reg_body(const EvalArgs& a, int block) {
    const int idx = block * 256 + threadIdx.x;
    if (idx >= (a.blist ? a.n_blist : a.n_branches) * a.K) return;
    const int b = a.blist ? a.blist[idx / a.K] : idx / a.K, l = idx % a.K;
    const double tb = a.t[b];
    T* out = static_cast<T*>(a.P) + ((size_t)b * a.K + l) * M * M;
    if (bad_length(tb)) {
#pragma unroll
        for (int e = 0; e < M * M; ++e) out[e] = T(NAN);
        return;
    }
    const double h = a.rates[l] * tb;
    const double* Qb = branch_q(a, b, M);
    double nrm = branch_qnorm(a, b) * h;
    int s = 0;
    while (nrm > 0.5 && s < 1100) { nrm *= 0.5; ++s; }
    const double hs = ldexp(h, -s);
    double A[M][M], G[M][M], W[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            A[i][j] = Qb[i * M + j] * hs;
            G[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int k = TAYLOR_DEG; k >= 2; --k) {
        matmul_reg<M>(A, G, W);
        const double inv = 1.0 / k;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) G[i][j] = ((i == j) ? 1.0 : 0.0) + W[i][j] * inv;
    }
    matmul_reg<M>(A, G, W);  // W = F
    for (int r = 0; r < s; ++r) {
        matmul_reg<M>(W, W, G);
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) W[i][j] = 2.0 * W[i][j] + G[i][j];
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) out[i * M + j] = T(((i == j) ? 1.0 : 0.0) + W[i][j]);
}

// One workgroup per (branch, category); matrices in LDS (larger M).
template <int M, typename T>
__device__ inline void pmat_lds_body(const EvalArgs& a, int block) {
    __shared__ double A[M * M], G[M * M], W[M * M];
    const int idx = block;
    const int b = a.blist ? a.blist[idx / a.K] : idx / a.K, l = idx % a.K;
    T* out = static_cast<T*>(a.P) + ((size_t)b * a.K + l) * M * M;
    if (!taylor_F_lds<M>(a, b, l, A, G, W)) {
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) out[e] = T(NAN);
        return;
    }
    for (int e = threadIdx.x; e < M * M; e += blockDim.x)
        out[e] = T(((e / M == e % M) ? 1.0 : 0.0) + W[e]);
}

// ---------------------------------------------------------------- post-order pass
//
// For each internal node k (children i, j), category l, pattern s:
//   p_k = (P_i p_i) o (P_j p_j)                  Eq. (postOrderPartialUpdate)
//   p~_k = p_k 2^-e, e = exponent of max_x p_k   exact rescaling
//   store m_k = P_k p~_k unless k is the root; at the root keep
//   pi^T p~_root                                 Eq. (rootInnerProduct)
// and the summed exponents of the pattern's column.

// p~_k of node k from its children's messages, with the exponent
// bookkeeping (esum, and the stored per-node exponents when kept).
// p = mi o mj rescaled by the exact power of two 2^-e that brings its
// largest entry into [1/2, 1); returns e (0 for an all-zero product).
template <int M, typename T>
__device__ inline int scaled_product(const T mi[M], const T mj[M], T p[M]) {
    T mx = T(0);
#pragma unroll
    for (int x = 0; x < M; ++x) {
        p[x] = mi[x] * mj[x];
        mx = fmax(mx, p[x]);
    }
    int e = 0;
    if (mx > T(0)) {
        e = exp_of(mx);
#pragma unroll
        for (int x = 0; x < M; ++x) p[x] = pow2_scale(p[x], -e);
    }
    return e;
}

template <int M, typename T>
__device__ inline void post_combine(const EvalArgs& a, int k, int tile, int ps, const T mi[M], const T mj[M],
                                    T p[M], int& esum) {
    const int e = scaled_product<M, T>(mi, mj, p);
    if (a.expo) {
        // per-node exponents for partial re-evaluation: a pass over some
        // nodes adds the change of each visited node's exponent
        int16_t* ex = a.expo + ((size_t)(k - a.n_tips) * a.n_tiles + tile) * TP + ps;
        if (a.expo_delta) esum += e - (int)*ex;
        else esum += e;
        *ex = (int16_t)e;
    } else {
        esum += e;
    }
}

template <int M, typename T>
__device__ inline void post_node(const EvalArgs& a, int4 nd, int l, int tile, int s, int ps,
                                 const ChildRaw<M, T>& ri, const ChildRaw<M, T>& rj, T pk, int& esum) {
    T mi[M], mj[M], p[M];
    child_finish<M, T>(a, nd.y, l, ri, mi);
    child_finish<M, T>(a, nd.z, l, rj, mj);
    const int k = nd.x;
    post_combine<M, T>(a, k, tile, ps, mi, mj, p, esum);
    if (k != a.root) {
        T mk[M];
        if constexpr (RowMat<M>::value) {
            row_matvec<M, T>(pk, p, mk);
        } else {
            const T* Pk = pmat_of<M, T>(a, k, l);
#pragma unroll
            for (int x = 0; x < M; ++x) {
                T acc = T(0);
#pragma unroll
                for (int y = 0; y < M; ++y) acc = fma(Pk[x * M + y], p[y], acc);
                mk[x] = acc;
            }
        }
        T* out = static_cast<T*>(a.msg) + vec_off(a, k, tile, M) + ps;
#pragma unroll
        for (int x = 0; x < M; ++x) out[x * TP] = mk[x];
    } else {
        double Lt = 0.0;
#pragma unroll
        for (int x = 0; x < M; ++x) Lt = fma(pientry<M>(a, x), (double)p[x], Lt);
        a.rootL[(size_t)l * a.S_pad + s] = Lt;
    }
}

// ---------------------------------------------------------------- clade walks
//
// Below the top of the tree each clade list is walked depth first with no
// workgroup barrier (the launches of their own are further below): entries
// come in post order (the child with more internal nodes first), so the
// message of the last finished node is the second child's and stays in
// registers, and a first child whose sibling is internal parks its message
// on the row's LDS stack (at most log2 of the clade size deep).  The
// pre-order walk takes the same entries backwards and passes q the same way.
// Pieces shared by the walks:

template <int M, typename T>
__device__ inline void stack_push(T* stk, int& sp, const T v[M]) {
#pragma unroll
    for (int x = 0; x < M; ++x) stk[(sp * M + x) * TP] = v[x];
    ++sp;
}
template <int M, typename T>
__device__ inline void stack_pop(T* stk, int& sp, T v[M]) {
    --sp;
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = stk[(sp * M + x) * TP];
}

// Tip message with a row-distributed P (pe = this lane's entry): the
// observed state's column, read from the lane holding entry (x, code);
// ambiguity codes (rare) sum the allowed columns, masks from the LDS copy.
template <int M, typename T>
__device__ inline void tip_message(unsigned code, T pe, const unsigned long long* lmask, T out[M]) {
    const int col = code < (unsigned)M ? (int)code : 0;
#pragma unroll
    for (int x = 0; x < M; ++x) out[x] = __shfl(pe, x * M + col, TP);
    if (__any(code >= (unsigned)M)) {
        T amb[M];
        row_masked_rows<M, T>(pe, lmask[code & 255u], amb);
        if (code >= (unsigned)M) {
#pragma unroll
            for (int x = 0; x < M; ++x) out[x] = amb[x];
        }
    }
}

// The clade walks issue every load of an entry whatever its children are
// (a tip child's message slot and an internal child's code read valid,
// unused addresses), so each entry has the same number of loads in flight
// and the wait before an entry's use counts only the loads issued after it,
// leaving the prefetched entries in flight.
template <int M, typename T>
struct ChildAll {
    T v[M];         // message of an internal child
    T pe;           // this lane's entry of the child's P
    unsigned code;  // tip code
};

template <int M, typename T>
__device__ inline void child_msg_all(const EvalArgs& a, int c, const ChildAll<M, T>& r,
                                     const unsigned long long* lmask, T out[M]) {
    if (c < a.n_tips) {
        tip_message<M, T>(r.code, r.pe, lmask, out);
    } else {
#pragma unroll
        for (int x = 0; x < M; ++x) out[x] = r.v[x];
    }
}

// Loads of one post-order clade entry: the children's codes and matrix
// entries and the node's own entry (internal children's messages are in
// registers or on the stack).
template <int M, typename T>
struct PostCladeRaw {
    unsigned code0, code1;
    T pe0, pe1, pk;
};

// Copy of the code -> state mask table in LDS (ambiguity codes).
__device__ inline void stage_masks(const EvalArgs& a, unsigned long long* lmask) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) lmask[i] = a.masks[i];
    __syncthreads();
}
// The same copy in two steps, for blocks of at least 256 threads: the load
// is issued early with the block's other loads, the store after them (the
// caller's barrier publishes the table).
__device__ inline unsigned long long mask_load(const EvalArgs& a) { return a.masks[min((int)threadIdx.x, 255)]; }
__device__ inline void mask_store(unsigned long long* lmask, unsigned long long v) {
    if (threadIdx.x < 256) lmask[threadIdx.x] = v;
}

// Level walk of the post-order pass over the schedule's levels (the whole
// tree, or the top above the clades): node slot ns of NS takes every NS-th
// node of a level; a barrier separates levels.
template <int M, typename T, int NS>
__device__ inline void post_levels(const EvalArgs& a, const int4* lds_sched, int l, int tile, int s, int ps, int ns,
                                   int& esum) {
    for (int h = 0; h < a.n_levels; ++h) {
        const int end = uniform_int(a.level_off, h + 1);
        int idx = uniform_int(a.level_off, h) + ns;
        if (idx < end) {
            // software pipeline: the next node's loads are issued before this
            // node's stores, so they never wait behind them
            int4 nd = sched_at(a, lds_sched, idx);
            ChildRaw<M, T> ri, rj;
            T pk = T(0);
            child_load<M, T>(a, nd.y, l, tile, s, ps, ri);
            child_load<M, T>(a, nd.z, l, tile, s, ps, rj);
            if constexpr (RowMat<M>::value)
                if (nd.x != a.root) pk = load_row_entry<M, T>(pmat_of<M, T>(a, nd.x, l), ps);
            while (true) {
                const int nidx = idx + NS;
                const bool more = nidx < end;
                int4 nn = nd;
                ChildRaw<M, T> ni, nj;
                T npk = T(0);
                if (more) {
                    nn = sched_at(a, lds_sched, nidx);
                    child_load<M, T>(a, nn.y, l, tile, s, ps, ni);
                    child_load<M, T>(a, nn.z, l, tile, s, ps, nj);
                    if constexpr (RowMat<M>::value)
                        if (nn.x != a.root) npk = load_row_entry<M, T>(pmat_of<M, T>(a, nn.x, l), ps);
                }
                post_node<M, T>(a, nd, l, tile, s, ps, ri, rj, pk, esum);
                if (!more) break;
                nd = nn;
                ri = ni;
                rj = nj;
                pk = npk;
                idx = nidx;
            }
        }
        __syncthreads();
    }
}

// The pattern's summed scale exponent of the tile's category: the NS slots'
// sums in slot order, plus the parts of a separate clade launch.
template <int NS>
__device__ inline void post_root_exponents(const EvalArgs& a, int l, int tile, int s, int ps, int ns, int esum) {
    __shared__ int red[NS][TP];
    red[ns][ps] = esum;
    __syncthreads();
    if (ns == 0) {
        int tot = 0;
        for (int i = 0; i < NS; ++i) tot += red[i][ps];
        // exponents summed by the separate clade launch, one part per workgroup
        for (int q = 0; q < a.n_cl_esum; ++q) tot += a.cl_esum[((size_t)q * a.n_tiles + tile) * TP + ps];
        if (a.expo_delta) a.rootE[(size_t)l * a.S_pad + s] += tot;
        else a.rootE[(size_t)l * a.S_pad + s] = tot;
    }
}

template <int M, typename T>
__device__ inline void post_body(const EvalArgs& a, int tile, int4* lds_sched) {
    constexpr int NS = post_slots<T>(M);
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int ps = threadIdx.x % TP, ns = threadIdx.x / TP;
    const int s = pb * TP + ps;
    stage_schedule(a, lds_sched);
    int esum = 0;
    post_levels<M, T, NS>(a, lds_sched, l, tile, s, ps, ns, esum);
    post_root_exponents<NS>(a, l, tile, s, ps, ns, esum);
}

template <int NT>
__device__ void finish_logl(const EvalArgs& a) {
    double acc = 0.0;
    int flag = 0;
    for (int pb = threadIdx.x; pb < a.n_pb; pb += NT) {
        acc += a.logl_part[pb];
        flag |= a.flag_part[pb];
    }
    __shared__ double red[NT];
    __shared__ int fred[NT];
    red[threadIdx.x] = acc;
    fred[threadIdx.x] = flag;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            fred[threadIdx.x] |= fred[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int f = fred[0];
        a.logL_out[0] = (f & 1) ? NAN : (f & 2) ? -INFINITY : red[0];
        a.status[0] = (f & 1) ? 1 : (f & 2) ? 2 : 0;
    }
}

// Forward-only calls: one block forms every part, then finishes.
constexpr int LOGL_THREADS = 1024;

__global__ void __launch_bounds__(LOGL_THREADS) logl_kernel(EvalArgs a) {
    const int ps = threadIdx.x % TP, row = threadIdx.x / TP;
    for (int pb = row; pb < a.n_pb; pb += LOGL_THREADS / TP)
        logl_block_part(a, pb, ps, site_likelihood(a, pb * TP + ps));
    __threadfence_block();
    __syncthreads();
    finish_logl<LOGL_THREADS>(a);
}

// ---------------------------------------------------------------- pre-order pass + gradient
//
// For each internal node k (children i, j; q_root = pi), category l,
// pattern s, and each child a with sibling b:
//   u_a = q~_k o m_b                          top-of-branch vector
//   r_a = (u_a^T Q m_a) / (u_a^T m_a)         Eq. (singleRateCaseGradient)
//   tile sum of w_s rho_{s,l} gamma_l r_a     Eq. (GradientWithGamma)
//   q_a = P_a^T u_a, rescaled, stored if a is internal   Eq. (preOrderUpdate)
// The numerator uses Q m_a = Q P_a p_a = P_a Q p_a, so q_a^T Q p_a is
// u_a^T Q m_a.

// HESS adds, for Eq. (Hessian) of Section 2.7 per site:
//   tile sum of w_s rho gamma^2 (u^T Q^2 m)/(u^T m)   -> partial2[tile][c]
//   rho gamma (u^T Q m)/(u^T m) for every pattern     -> r1[c][l][s]
// so d2 logL/dt_c^2 = sum partial2 - sum_s w_s (sum_l r1)^2.
// u_a^T m_a is the same for both children of a node (sum_x q_x m_i,x m_j,x),
// so it is formed once per node and its reciprocal (0 when the sum is not
// positive: no contribution) serves both children's ratios.
// (FP32 partials: the hardware FP32 reciprocal, within about 1 ulp, far
// inside that path's accuracy.)
template <int M, typename T>
__device__ inline double node_rden(const T u[M], const T mown[M]) {
    T den = T(0);
#pragma unroll
    for (int x = 0; x < M; ++x) den = fma(u[x], mown[x], den);
    if constexpr (sizeof(T) == 4) return (den > T(0)) ? (double)__builtin_amdgcn_rcpf(den) : 0.0;
    return (den > T(0)) ? 1.0 / (double)den : 0.0;
}

// Gradient term (and, HESS, Hessian term) of child c with its
// top-of-branch vector u and own message mown; rden from node_rden.  Leaves
// this lane's terms in term / term2 for the caller's row sums.
template <int M, typename T, bool HESS, bool NH>
__device__ inline void child_terms(const EvalArgs& a, int c, int l, int s, const Coef& cf, const T u[M],
                                   const T mown[M], double rden, double& term, double& term2) {
    T num = T(0), num2 = T(0);
    if constexpr (!NH) {
        // the model's Q (kernel arguments for small M)
#pragma unroll
        for (int x = 0; x < M; ++x) {
            T qm = T(0);
#pragma unroll
            for (int y = 0; y < M; ++y) qm = fma(T(qentry<M>(a, x * M + y)), mown[y], qm);
            num = fma(u[x], qm, num);
            if constexpr (HESS) {
                T q2m = T(0);
#pragma unroll
                for (int y = 0; y < M; ++y) q2m = fma(T(q2entry<M>(a, x * M + y)), mown[y], q2m);
                num2 = fma(u[x], q2m, num2);
            }
        }
    } else {
        // non-homogeneous model: Q and Q^2 of branch c
        const double* Qc = a.Qm + (size_t)a.branch_model[c] * M * M;
        const double* Q2c = a.Q2m + (size_t)a.branch_model[c] * M * M;
#pragma unroll
        for (int x = 0; x < M; ++x) {
            T qm = T(0);
#pragma unroll
            for (int y = 0; y < M; ++y) qm = fma(T(Qc[x * M + y]), mown[y], qm);
            num = fma(u[x], qm, num);
            if constexpr (HESS) {
                T q2m = T(0);
#pragma unroll
                for (int y = 0; y < M; ++y) q2m = fma(T(Q2c[x * M + y]), mown[y], q2m);
                num2 = fma(u[x], q2m, num2);
            }
        }
    }
    const double ratio = (double)num * rden;
    term = (cf.g > 0.0) ? cf.g * ratio : 0.0;
    if constexpr (HESS) {
        const double ratio2 = (double)num2 * rden;
        term2 = (cf.h > 0.0) ? cf.h * ratio2 : 0.0;
        a.r1[((size_t)c * a.K + l) * a.S_pad + s] = (cf.nw > 0.0) ? cf.nw * ratio : 0.0;
    }
}

// q~_c = P_c^T u of an internal child c, rescaled by an exact power of two
// (pc: this lane's entry of the row-distributed P_c for small M).
template <int M, typename T>
__device__ inline void child_q(const EvalArgs& a, int c, int l, T pc, const T u[M], T qout[M]) {
    T qc[M];
    if constexpr (RowMat<M>::value) {
        row_matvec_t<M, T>(pc, u, qc);
    } else {
        const T* Pc = pmat_of<M, T>(a, c, l);
#pragma unroll
        for (int y = 0; y < M; ++y) {
            T acc = T(0);
#pragma unroll
            for (int x = 0; x < M; ++x) acc = fma(Pc[x * M + y], u[x], acc);
            qc[y] = acc;
        }
    }
    T mx = T(0);
#pragma unroll
    for (int y = 0; y < M; ++y) mx = fmax(mx, qc[y]);
    const int e = (mx > T(0)) ? exp_of(mx) : 0;
#pragma unroll
    for (int y = 0; y < M; ++y) qout[y] = pow2_scale(qc[y], -e);
}

// Both for child c: the terms (child_terms) and, when c is internal, q~_c in
// qout (returns true).
template <int M, typename T, bool HESS, bool NH>
__device__ inline bool pre_child_core(const EvalArgs& a, int c, int l, int tile, int s, int ps, const Coef& cf,
                                      const T u[M], const T mown[M], double rden, T pc, double& term,
                                      double& term2, T qout[M]) {
    child_terms<M, T, HESS, NH>(a, c, l, s, cf, u, mown, rden, term, term2);
    if (c >= a.n_tips) {
        child_q<M, T>(a, c, l, pc, u, qout);
        return true;
    }
    return false;
}

// Whether a node's two children reduce their terms together.
template <bool HESS, bool NH>
constexpr bool PAIR_TERMS = !HESS && !NH;

// FP32 partials: the row sums in FP32 (single-precision DPP adds; the
// terms are rounded to FP32 first, far inside that path's accuracy).
template <int CTRL>
__device__ inline float dpp32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ inline float pair_sum16f(float a, float b, bool upper) {
    float v = (upper ? b : a) + dpp32<0x128>(upper ? a : b);  // row_ror 8
    v += dpp32<0x141>(v);                                      // row_half_mirror
    v += dpp32<0x4E>(v);                                       // quad_perm [2, 3, 0, 1]
    v += dpp32<0xB1>(v);                                       // quad_perm [1, 0, 3, 2]
    return v;
}
template <typename T>
__device__ inline double pair_sum_t(double a, double b, bool upper) {
    if constexpr (sizeof(T) == 4) return (double)pair_sum16f((float)a, (float)b, upper);
    return pair_sum16(a, b, upper);
}

// Tile sum of one child's term(s), right after its core step.  Lane 0 of
// pair_sum16(t, t) depends only on the lower half's association, which is
// the upper half's too, so every variant forms the same bits for a branch.
template <bool HESS, typename T>
__device__ inline void store_terms(const EvalArgs& a, int tile, int ps, int c, double t, double h) {
    const size_t at = (size_t)tile * a.n_branches + c;
    t = pair_sum_t<T>(t, t, ps >= 8);
    if (ps == 0) a.partial[at] = t;
    if constexpr (HESS) {
        h = pair_sum_t<T>(h, h, ps >= 8);
        if (ps == 0) a.partial2[at] = h;
    }
}

// Tile sums of both children's terms (Eq. GradientWithGamma; HESS: the
// Section 2.7 term too), reduced together over the row's 16 patterns and
// stored by lane 0 (first child) and lane 8 (second child) of the row.
template <bool HESS, typename T>
__device__ inline void store_pair_terms(const EvalArgs& a, int tile, int ps, int4 nd, double t0, double t1,
                                        double h0, double h1) {
    const size_t at = (size_t)tile * a.n_branches + (ps < 8 ? nd.y : nd.z);
    const double t = pair_sum_t<T>(t0, t1, ps >= 8);
    if ((ps & 7) == 0) a.partial[at] = t;
    if constexpr (HESS) {
        const double h = pair_sum_t<T>(h0, h1, ps >= 8);
        if ((ps & 7) == 0) a.partial2[at] = h;
    }
}

// q~_c goes to LDS (lds_dst) or to memory
template <int M, typename T>
__device__ inline void pre_store_q(const EvalArgs& a, int c, int tile, int ps, const T qc[M], T* lds_dst) {
    T* out = lds_dst ? lds_dst : static_cast<T*>(a.qv) + vec_off(a, c, tile, M) + ps;
#pragma unroll
    for (int y = 0; y < M; ++y) out[y * TP] = qc[y];
}

// Loads of one pre-order node: q of the node, both children's messages and,
// for small M, the children's own matrix entries.
template <int M, typename T>
struct PreRaw {
    T q[M];
    ChildRaw<M, T> ri, rj;
    T pi_, pj_;
};

// with_q = false leaves q to the caller (top region: LDS or pi)
template <int M, typename T>
__device__ inline void pre_load(const EvalArgs& a, int4 nd, int l, int tile, int s, int ps, PreRaw<M, T>& r,
                                bool with_q = true) {
    if (!with_q) {
    } else if (nd.x == a.root) {
#pragma unroll
        for (int x = 0; x < M; ++x) r.q[x] = T(pientry<M>(a, x));
    } else {
        const T* src = static_cast<const T*>(a.qv) + vec_off(a, nd.x, tile, M) + ps;
#pragma unroll
        for (int x = 0; x < M; ++x) r.q[x] = src[x * TP];
    }
    child_load<M, T>(a, nd.y, l, tile, s, ps, r.ri);
    child_load<M, T>(a, nd.z, l, tile, s, ps, r.rj);
    r.pi_ = r.pj_ = T(0);
    if constexpr (RowMat<M>::value) {
        if (nd.y >= a.n_tips) r.pi_ = load_row_entry<M, T>(pmat_of<M, T>(a, nd.y, l), ps);
        if (nd.z >= a.n_tips) r.pj_ = load_row_entry<M, T>(pmat_of<M, T>(a, nd.z, l), ps);
    }
}

// top == nullptr: q of internal children goes to HBM; otherwise children in
// the top region keep q in LDS only (it is consumed inside the region)
template <int M, typename T, bool HESS, bool NH>
__device__ inline void pre_node(const EvalArgs& a, int4 nd, int l, int tile, int s, int ps, const Coef& cf,
                                const T q[M], const PreRaw<M, T>& r, T* top) {
    T mi[M], mj[M];
    child_finish<M, T>(a, nd.y, l, r.ri, mi);
    child_finish<M, T>(a, nd.z, l, r.rj, mj);
    // a tip child's own matrix entry travels in its raw message slot
    const T pi_ = (nd.y < a.n_tips) ? r.ri.v[0] : r.pi_;
    const T pj_ = (nd.z < a.n_tips) ? r.rj.v[0] : r.pj_;
    T* di = nullptr;
    T* dj = nullptr;
    if (top) {
        if (const int si = rslot(nd.w, 1)) di = top_vec<M, T>(top, si, ps);
        if (const int sj = rslot(nd.w, 2)) dj = top_vec<M, T>(top, sj, ps);
    }
    T ui[M], uj[M];
#pragma unroll
    for (int x = 0; x < M; ++x) {
        ui[x] = q[x] * mj[x];
        uj[x] = q[x] * mi[x];
    }
    const double rden = node_rden<M, T>(ui, mi);
    double t0, t1, h0 = 0.0, h1 = 0.0;
    T qi[M], qj[M];
    const bool ini = pre_child_core<M, T, HESS, NH>(a, nd.y, l, tile, s, ps, cf, ui, mi, rden, pi_, t0, h0, qi);
    if constexpr (!PAIR_TERMS<HESS, NH>) store_terms<HESS, T>(a, tile, ps, nd.y, t0, h0);
    const bool inj = pre_child_core<M, T, HESS, NH>(a, nd.z, l, tile, s, ps, cf, uj, mj, rden, pj_, t1, h1, qj);
    if constexpr (!PAIR_TERMS<HESS, NH>) store_terms<HESS, T>(a, tile, ps, nd.z, t1, h1);
    else store_pair_terms<HESS, T>(a, tile, ps, nd, t0, t1, h0, h1);
    if (ini) pre_store_q<M, T>(a, nd.y, tile, ps, qi, di);
    if (inj) pre_store_q<M, T>(a, nd.z, tile, ps, qj, dj);
}

// Clade part of the pre-order pass (after the top): q of a clade root comes
// from memory, q of a second child (or of a first child with a tip sibling)
// from registers, q of a first child with an internal sibling from the
// stack.  CLADE_DEPTH entries are in flight: an entry's loads are issued
// CLADE_DEPTH - 1 entries before it is processed.
#ifndef PG_CLADE_DEPTH
#define PG_CLADE_DEPTH 2
#endif
constexpr int CLADE_DEPTH = PG_CLADE_DEPTH;

template <int M, typename T>
struct PreCladeRaw {
    T q[M];  // clade root: q from memory
    ChildAll<M, T> c0, c1;
};

template <int M, typename T, bool HESS, bool NH>
__device__ inline void pre_clade_node(const EvalArgs& a, int4 nd, int l, int tile, int s, int ps, const Coef& cf,
                                      const PreCladeRaw<M, T>& r, const unsigned long long* lmask, T acc[M],
                                      T* stk, int& sp) {
    T q[M];
    if (nd.w & CL_ROOT) {
#pragma unroll
        for (int x = 0; x < M; ++x) q[x] = r.q[x];
    } else if (nd.w & CL_STACK) {
        stack_pop<M, T>(stk, sp, q);
    } else {
#pragma unroll
        for (int x = 0; x < M; ++x) q[x] = acc[x];
    }
    T m0[M], m1[M], q0[M], q1[M];
    child_msg_all<M, T>(a, nd.y, r.c0, lmask, m0);
    child_msg_all<M, T>(a, nd.z, r.c1, lmask, m1);
    T u0[M], u1[M];
#pragma unroll
    for (int x = 0; x < M; ++x) {
        u0[x] = q[x] * m1[x];
        u1[x] = q[x] * m0[x];
    }
    const double rden = node_rden<M, T>(u0, m0);
    double t0, t1, h0 = 0.0, h1 = 0.0;
    const bool in0 = pre_child_core<M, T, HESS, NH>(a, nd.y, l, tile, s, ps, cf, u0, m0, rden, r.c0.pe, t0, h0, q0);
    // the Hessian and per-branch-model variants reduce each child at once
    // (holding both children's terms spills them at FP32's register budget)
    if constexpr (!PAIR_TERMS<HESS, NH>) store_terms<HESS, T>(a, tile, ps, nd.y, t0, h0);
    const bool in1 = pre_child_core<M, T, HESS, NH>(a, nd.z, l, tile, s, ps, cf, u1, m1, rden, r.c1.pe, t1, h1, q1);
    if constexpr (!PAIR_TERMS<HESS, NH>) store_terms<HESS, T>(a, tile, ps, nd.z, t1, h1);
    else store_pair_terms<HESS, T>(a, tile, ps, nd, t0, t1, h0, h1);
    // the second child's subtree comes next, then the first child's
    if (in1) {
        if (in0) stack_push<M, T>(stk, sp, q0);
#pragma unroll
        for (int x = 0; x < M; ++x) acc[x] = q1[x];
    } else if (in0) {
#pragma unroll
        for (int x = 0; x < M; ++x) acc[x] = q0[x];
    }
}

// NH: non-homogeneous model (Q of each child's branch from a table); a
// separate instantiation, so the homogeneous kernel keeps Q in its arguments.
template <int M, typename T, bool HESS, bool NH>
__device__ inline void pre_body(const EvalArgs& a, int tile, int4* lds_sched) {
    constexpr int NS = pre_slots<T>(M);
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int ps = threadIdx.x % TP, ns = threadIdx.x / TP;
    const int s = pb * TP + ps;
    // rho_{s,l} gamma_l w_s from the per-category root values
    Coef cf;
    {
        const SiteLik r = site_likelihood(a, s);
        cf = coef_of(a, l, s, r);
        // the category-0 tile of each pattern block also forms its logL part
        if (l == 0 && ns == 0) logl_block_part(a, pb, ps, r);
    }
    stage_schedule(a, lds_sched);
    T* top = top_buffer<T>(a, lds_sched);
    // top region first: each slot issues its next level's loads (children
    // messages of the post-order pass) before the LDS-only barrier; the last
    // region level ends with a full barrier so the q written to HBM for the
    // levels below is visible
    if (a.top_level < a.n_levels) {
        int h = a.n_levels - 1;
        int idx = uniform_int(a.level_off, h) + ns;
        bool have = idx < uniform_int(a.level_off, h + 1);
        int4 nd = make_int4(0, 0, 0, 0);
        PreRaw<M, T> cur;
        if (have) {
            nd = sched_at(a, lds_sched, idx);
            pre_load<M, T>(a, nd, l, tile, s, ps, cur, false);
        }
        for (; h >= a.top_level; --h) {
            const int h2 = h - 1;
            const int hc = max(h2, a.top_level);
            const int idx2 = (h2 >= a.top_level) ? uniform_int(a.level_off, hc) + ns : 0;
            const bool have2 = h2 >= a.top_level && idx2 < uniform_int(a.level_off, hc + 1);
            int4 nd2 = make_int4(0, 0, 0, 0);
            PreRaw<M, T> nxt;
            if (have2) {
                nd2 = sched_at(a, lds_sched, idx2);
                pre_load<M, T>(a, nd2, l, tile, s, ps, nxt, false);
            }
            if (have) {
                T q[M];
                if (nd.x == a.root) {
#pragma unroll
                    for (int x = 0; x < M; ++x) q[x] = T(pientry<M>(a, x));
                } else {
                    const T* src = top_vec<M, T>(top, rslot(nd.w, 0), ps);
#pragma unroll
                    for (int x = 0; x < M; ++x) q[x] = src[x * TP];
                }
                pre_node<M, T, HESS, NH>(a, nd, l, tile, s, ps, cf, q, cur, top);
            }
            if (h > a.top_level) lds_barrier();
            else __syncthreads();
            have = have2;
            nd = nd2;
            cur = nxt;
        }
    }
    // wide levels: several nodes per slot, software-pipelined
    for (int h = a.top_level - 1; h >= 0; --h) {
        const int end = uniform_int(a.level_off, h + 1);
        int idx = uniform_int(a.level_off, h) + ns;
        if (idx < end) {
            int4 nd = sched_at(a, lds_sched, idx);
            PreRaw<M, T> cur;
            pre_load<M, T>(a, nd, l, tile, s, ps, cur);
            while (true) {
                const int nidx = idx + NS;
                const bool more = nidx < end;
                int4 nn = nd;
                PreRaw<M, T> nxt;
                if (more) {
                    nn = sched_at(a, lds_sched, nidx);
                    pre_load<M, T>(a, nn, l, tile, s, ps, nxt);
                }
                pre_node<M, T, HESS, NH>(a, nd, l, tile, s, ps, cf, cur.q, cur, nullptr);
                if (!more) break;
                nd = nn;
                cur = nxt;
                idx = nidx;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- clade walks, one list per wave
//
// The clade walks as launches of their own (the top levels run in the
// post-order launch after them and in the pre-order launch before them):
// here a wavefront walks one clade list for four tiles at once, one tile per
// 16-lane row, instead of four lists for one tile.  Every entry, and with it
// whether a child is a tip or internal, is then the same across the
// wavefront: the entries are read into scalar registers, the tip / internal
// and stack / register choices are scalar branches that run only the path
// taken, and node addresses are a scalar base plus a per-lane offset that
// never changes during the walk.  The per-lane arithmetic is that of the
// combined kernels above, so both give the same bits.
//
// A workgroup holds CW_WAVES lists of one group of four tiles.  Tiles are
// grouped in pattern-block-major order (t' = pb K + l; with K = 4 a group is
// the four rate categories of one pattern block); a short last group
// repeats its last tile, whose rows then compute and store the same values.
constexpr int CW_ROWS = 64 / TP;  // tiles per group (rows per wavefront)

struct CwLane {
    int tile, l, pb, s, ps;
    unsigned vec;  // tile * M * TP + ps: this lane's element of a node's block
    unsigned pe;   // l * M * M + ps: this lane's entry of a branch's matrices
};

template <int M>
__device__ inline CwLane cw_lane(const EvalArgs& a, int group) {
    const int lane = threadIdx.x % 64, row = lane / TP;
    CwLane ln;
    ln.ps = lane % TP;
    const int tp = min(group * CW_ROWS + row, a.n_tiles - 1);
    ln.pb = tp / a.K;
    ln.l = tp % a.K;
    ln.tile = ln.l * a.n_pb + ln.pb;
    ln.s = ln.pb * TP + ln.ps;
    ln.vec = (unsigned)(ln.tile * (M * TP) + ln.ps);
    ln.pe = (unsigned)(ln.l * (M * M) + ln.ps);
    return ln;
}

// Element offsets in 32 bits (fewer scalar instructions per address): the
// launcher takes these walks only when every vector buffer holds fewer than
// 2^31 elements.
template <int M, typename T>
__device__ inline const T* node_block(const EvalArgs& a, const void* base, int node) {
    return static_cast<const T*>(base) + (unsigned)((node - a.n_tips) * (a.n_tiles * (M * TP)));
}
template <int M, typename T>
__device__ inline const T* branch_mats(const EvalArgs& a, int b) {
    return static_cast<const T*>(a.P) + (unsigned)(b * a.K * (M * M));
}
__device__ inline const uint8_t* code_row(const EvalArgs& a, int tip) {
    return a.codes + (unsigned)(tip * a.S_pad);
}

template <int M, typename T>
__device__ inline void post_clade_load_u(const EvalArgs& a, int4 nd, const CwLane& ln, PostCladeRaw<M, T>& r) {
    r.code0 = code_row(a, nd.y < a.n_tips ? nd.y : 0)[ln.s];
    r.code1 = code_row(a, nd.z < a.n_tips ? nd.z : 0)[ln.s];
    r.pe0 = branch_mats<M, T>(a, nd.y)[ln.pe];
    r.pe1 = branch_mats<M, T>(a, nd.z)[ln.pe];
    r.pk = branch_mats<M, T>(a, nd.x)[ln.pe];
}

template <int M, typename T>
__device__ inline void post_clades_u(const EvalArgs& a, int list, const CwLane& ln, T* stk,
                                     const unsigned long long* lmask, int& esum) {
    const int beg = uniform_int(a.cl_post_off, list), end = uniform_int(a.cl_post_off, list + 1);
    if (beg >= end) return;
    int sp = 0;
    T acc[M];
#pragma unroll
    for (int x = 0; x < M; ++x) acc[x] = T(0);
    auto entry = [&](int i) { return uniform_entry(a.cl_post, min(i, end - 1)); };
    int4 nd = entry(beg);
    int4 nn = entry(beg + 1);
    PostCladeRaw<M, T> cur;
    post_clade_load_u<M, T>(a, nd, ln, cur);
    for (int i = beg;; ++i) {
        const int4 n2 = entry(i + 2);
        PostCladeRaw<M, T> nxt;
        post_clade_load_u<M, T>(a, nn, ln, nxt);
        T m0[M], m1[M], p[M], mk[M];
        if (nd.y < a.n_tips) {
            tip_message<M, T>(cur.code0, cur.pe0, lmask, m0);
        } else if (nd.z < a.n_tips) {
#pragma unroll
            for (int x = 0; x < M; ++x) m0[x] = acc[x];
        } else {
            stack_pop<M, T>(stk, sp, m0);
        }
        if (nd.z < a.n_tips) {
            tip_message<M, T>(cur.code1, cur.pe1, lmask, m1);
        } else {
#pragma unroll
            for (int x = 0; x < M; ++x) m1[x] = acc[x];
        }
        post_combine<M, T>(a, nd.x, ln.tile, ln.ps, m0, m1, p, esum);
        row_matvec<M, T>(cur.pk, p, mk);
        T* out = const_cast<T*>(node_block<M, T>(a, a.msg, nd.x)) + ln.vec;
#pragma unroll
        for (int x = 0; x < M; ++x) out[x * TP] = mk[x];
        if (nd.w & CL_STACK) {
            stack_push<M, T>(stk, sp, mk);
        } else {
#pragma unroll
            for (int x = 0; x < M; ++x) acc[x] = mk[x];
        }
        if (i + 1 >= end) break;
        nd = nn;
        nn = n2;
        cur = nxt;
    }
}

template <int M, typename T>
__device__ inline void child_load_all_u(const EvalArgs& a, int c, const CwLane& ln, ChildAll<M, T>& r) {
    const bool tip = c < a.n_tips;
    const T* src = node_block<M, T>(a, a.msg, tip ? a.n_tips : c) + ln.vec;
#pragma unroll
    for (int x = 0; x < M; ++x) r.v[x] = src[x * TP];
    r.code = code_row(a, tip ? c : 0)[ln.s];
    r.pe = branch_mats<M, T>(a, c)[ln.pe];
}

template <int M, typename T>
__device__ inline void pre_clade_load_u(const EvalArgs& a, int4 nd, const CwLane& ln, PreCladeRaw<M, T>& r) {
    const T* src = node_block<M, T>(a, a.qv, (nd.w & CL_ROOT) ? nd.x : a.n_tips) + ln.vec;
#pragma unroll
    for (int x = 0; x < M; ++x) r.q[x] = src[x * TP];
    child_load_all_u<M, T>(a, nd.y, ln, r.c0);
    child_load_all_u<M, T>(a, nd.z, ln, r.c1);
}

template <int M, typename T, bool HESS, bool NH>
__device__ inline void pre_clades_u(const EvalArgs& a, int list, const CwLane& ln, const Coef& cf, T* stk,
                                    const unsigned long long* lmask) {
    const int beg = uniform_int(a.cl_pre_off, list), end = uniform_int(a.cl_pre_off, list + 1);
    const int n = end - beg;
    if (n <= 0) return;
    int sp = 0;
    T acc[M];
#pragma unroll
    for (int x = 0; x < M; ++x) acc[x] = T(0);
    // entry i of the walk is list entry end - 1 - i; entries past the end
    // reload the last one, so every step issues the same loads
    auto entry = [&](int i) { return uniform_entry(a.cl_pre, end - 1 - min(i, n - 1)); };
    int4 nd[CLADE_DEPTH];
    PreCladeRaw<M, T> raw[CLADE_DEPTH];
#pragma unroll
    for (int j = 0; j < CLADE_DEPTH; ++j) {
        nd[j] = entry(j);
        pre_clade_load_u<M, T>(a, nd[j], ln, raw[j]);
    }
    int4 ne = entry(CLADE_DEPTH);
    for (int i0 = 0; i0 < n; i0 += CLADE_DEPTH) {
#pragma unroll
        for (int j = 0; j < CLADE_DEPTH; ++j) {
            if (i0 + j < n)
                pre_clade_node<M, T, HESS, NH>(a, nd[j], ln.l, ln.tile, ln.s, ln.ps, cf, raw[j], lmask, acc, stk, sp);
            const int4 ne2 = entry(i0 + j + CLADE_DEPTH + 1);
            nd[j] = ne;
            pre_clade_load_u<M, T>(a, nd[j], ln, raw[j]);
            ne = ne2;
        }
    }
}

// LDS stack of this thread's row (wavefront w, row r: slot w * CW_ROWS + r).
template <int M, typename T>
__device__ inline T* cw_stack(const EvalArgs& a, T* base) {
    const int slot = threadIdx.x / TP;
    return base + (size_t)slot * a.cl_depth * (M * TP) + threadIdx.x % TP;
}

template <int M, typename T>
__device__ inline void post_clade_body(const EvalArgs& a, int block, int4* lds_dyn) {
    constexpr int NQ = post_slots<T>(M) / CW_WAVES;
    const int group = block / NQ, q = block % NQ;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const CwLane ln = cw_lane<M>(a, group);
    __shared__ unsigned long long lmask[256];
    stage_masks(a, lmask);
    int esum = 0;
    post_clades_u<M, T>(a, __builtin_amdgcn_readfirstlane(q * CW_WAVES + wave), ln,
                        cw_stack<M, T>(a, reinterpret_cast<T*>(lds_dyn)), lmask, esum);
    // this workgroup's part of each pattern's exponent sum, lists in order
    __shared__ int red[CW_WAVES][64];
    red[wave][lane] = esum;
    __syncthreads();
    if (wave == 0) {
        int tot = 0;
#pragma unroll
        for (int w = 0; w < CW_WAVES; ++w) tot += red[w][lane];
        a.cl_esum[((size_t)q * a.n_tiles + ln.tile) * TP + ln.ps] = tot;
    }
}

template <int M, typename T, bool HESS, bool NH>
__device__ inline void pre_clade_body(const EvalArgs& a, int block, int4* lds_dyn) {
    constexpr int NQ = pre_slots<T>(M) / CW_WAVES;
    const int group = block / NQ, q = block % NQ;
    const int wave = threadIdx.x / 64;
    const CwLane ln = cw_lane<M>(a, group);
    static_assert(CW_WAVES * 64 >= 256, "one mask per thread");
    SiteVals sv;
    site_vals_load(a, ln.l, ln.s, sv);
    const unsigned long long mv = mask_load(a);
    SiteLik r;
    const Coef cf = site_coef(a, ln.l, ln.s, sv, r);
    __shared__ unsigned long long lmask[256];
    mask_store(lmask, mv);
    __syncthreads();
    pre_clades_u<M, T, HESS, NH>(a, __builtin_amdgcn_readfirstlane(q * CW_WAVES + wave), ln, cf,
                                 cw_stack<M, T>(a, reinterpret_cast<T*>(lds_dyn)), lmask);
}

// Single evaluation (block = blockIdx.x) and batched entries (map[blockIdx.x]
// = {request, block}) of the clade launches; one block map serves both
// passes, whose list counts agree for small M.
static_assert(post_slots<double>(4) == pre_slots<double>(4) && post_slots<float>(4) == pre_slots<float>(4),
              "the post- and pre-order clade launches share their block map");

template <int M, typename T>
__global__ void __launch_bounds__(CW_WAVES * 64) __attribute__((amdgpu_waves_per_eu(RowMat<M>::value ? 4 : 1)))
post_clade_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    post_clade_body<M, T>(a, blockIdx.x, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(CW_WAVES * 64) __attribute__((amdgpu_waves_per_eu(RowMat<M>::value ? 4 : 1)))
post_clade_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    post_clade_body<M, T>(reqs[m.x], m.y, lds_dyn);
}

template <int M, typename T, bool HESS, bool NH>
__global__ void __launch_bounds__(CW_WAVES * 64) __attribute__((amdgpu_waves_per_eu(pre_waves<T>(M))))
pre_clade_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    pre_clade_body<M, T, HESS, NH>(a, blockIdx.x, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(CW_WAVES * 64) __attribute__((amdgpu_waves_per_eu(pre_waves<T>(M))))
pre_clade_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    pre_clade_body<M, T, false, false>(reqs[m.x], m.y, lds_dyn);
}

// ---------------------------------------------------------------- top levels next to the clade launches
//
// With the clade walks in launches of their own, the levels above the clades
// are a short chain of narrow levels, and every value they read from memory
// was written by an earlier launch: the clade roots' messages, the tips'
// codes, the branch matrices and, in the pre-order pass, the post-order
// messages.  Only the top nodes' own results pass from level to level
// (messages upwards, q downwards), and those stay in the top region in LDS.
// So each row issues the loads of all its top nodes at the start and waits
// for them once; the levels are then separated by LDS-only barriers, and no
// global store is waited for before the launch ends.  (In the level walk a
// level's loads wait behind the previous level's stores, which makes every
// level as long as a memory round trip.)
//
// Top node i (schedule order, levels in order) goes to row i % NS.  A level
// of the top region holds at most NS nodes, so they are on different rows,
// and a row holds at most TOP_J nodes (the launcher checks both).  The
// per-lane arithmetic is that of the level walk, so both give the same bits.

template <int M, typename T>
struct TopRaw {
    int4 nd;  // {node, child 0, child 1, region slots}
    ChildAll<M, T> c0, c1;
    T pk;  // post order: this lane's entry of the node's own matrix
};

template <int M>
__device__ inline CwLane top_lane(const EvalArgs& a, int tile) {
    CwLane ln;
    ln.tile = tile;
    ln.l = tile / a.n_pb;
    ln.pb = tile % a.n_pb;
    ln.ps = threadIdx.x % TP;
    ln.s = ln.pb * TP + ln.ps;
    ln.vec = (unsigned)(tile * (M * TP) + ln.ps);
    ln.pe = (unsigned)(ln.l * (M * M) + ln.ps);
    return ln;
}

// A child's loads; from_mem = false reads a valid, unused message slot in
// place of the child's (tips, and region children of the post-order pass,
// whose messages this launch forms).
template <int M, typename T>
__device__ inline void top_child_load(const EvalArgs& a, int c, bool from_mem, const CwLane& ln,
                                      ChildAll<M, T>& r) {
    const T* src = node_block<M, T>(a, a.msg, (c >= a.n_tips && from_mem) ? c : a.n_tips) + ln.vec;
#pragma unroll
    for (int x = 0; x < M; ++x) r.v[x] = src[x * TP];
    r.code = code_row(a, c < a.n_tips ? c : 0)[ln.s];
    r.pe = branch_mats<M, T>(a, c)[ln.pe];
}

// The loads of top node i; a row without an i-th node loads another node's
// (valid, unused).
template <int M, typename T, bool POST>
__device__ inline void top_load(const EvalArgs& a, int i, const CwLane& ln, TopRaw<M, T>& r) {
    r.nd = a.sched[min(max(i, 0), a.n_sched - 1)];
    top_child_load<M, T>(a, r.nd.y, !POST || rslot(r.nd.w, 1) == 0, ln, r.c0);
    top_child_load<M, T>(a, r.nd.z, !POST || rslot(r.nd.w, 2) == 0, ln, r.c1);
    r.pk = T(0);
    if constexpr (POST) r.pk = branch_mats<M, T>(a, r.nd.x == a.root ? 0 : r.nd.x)[ln.pe];
}

// A row's nodes are taken in order from raw[0]; after each, the rest move
// down one place (constant indices only: an indexed register array would
// live in scratch memory).
template <int M, typename T>
__device__ inline void top_shift(TopRaw<M, T> (&raw)[TOP_J]) {
#pragma unroll
    for (int k = 0; k + 1 < TOP_J; ++k) raw[k] = raw[k + 1];
}

template <int M, typename T>
__device__ inline void top_vec_load(const T* top, int slot, int ps, T v[M]) {
    const T* src = top_vec<M, T>(const_cast<T*>(top), slot, ps);
#pragma unroll
    for (int x = 0; x < M; ++x) v[x] = src[x * TP];
}

template <int M, typename T>
__device__ inline void post_top_body(const EvalArgs& a, int tile, T* top) {
    constexpr int NS = post_slots<T>(M);
    const int row = threadIdx.x / TP;
    const CwLane ln = top_lane<M>(a, tile);
    TopRaw<M, T> raw[TOP_J];
#pragma unroll
    for (int j = 0; j < TOP_J; ++j) top_load<M, T, true>(a, row + j * NS, ln, raw[j]);
    // the clade launch's exponent parts of the pattern (row 0 adds them)
    constexpr int NQ = NS / CW_WAVES;
    int parts[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        parts[q] = a.cl_esum[((size_t)min(q, a.n_cl_esum - 1) * a.n_tiles + tile) * TP + ln.ps];
    __shared__ unsigned long long lmask[256];
    stage_masks(a, lmask);  // its barrier also waits for the loads above
    int esum = 0, j = 0;
    for (int h = 0; h < a.n_levels; ++h) {
        // this row's next node (row + j NS, in raw[0]) lies on level h when it
        // precedes the next level
        if (j < TOP_J && row + j * NS < uniform_int(a.level_off, h + 1)) {
            const TopRaw<M, T>& r = raw[0];
            const int4 nd = r.nd;
            T m0[M], m1[M], p[M];
            if (const int s0 = rslot(nd.w, 1)) top_vec_load<M, T>(top, s0, ln.ps, m0);
            else child_msg_all<M, T>(a, nd.y, r.c0, lmask, m0);
            if (const int s1 = rslot(nd.w, 2)) top_vec_load<M, T>(top, s1, ln.ps, m1);
            else child_msg_all<M, T>(a, nd.z, r.c1, lmask, m1);
            esum += scaled_product<M, T>(m0, m1, p);
            if (nd.x != a.root) {
                T mk[M];
                row_matvec<M, T>(r.pk, p, mk);
                T* out = const_cast<T*>(node_block<M, T>(a, a.msg, nd.x)) + ln.vec;
                T* keep = top_vec<M, T>(top, rslot(nd.w, 0), ln.ps);
#pragma unroll
                for (int x = 0; x < M; ++x) {
                    out[x * TP] = mk[x];
                    keep[x * TP] = mk[x];
                }
            } else {
                double Lt = 0.0;
#pragma unroll
                for (int x = 0; x < M; ++x) Lt = fma(pientry<M>(a, x), (double)p[x], Lt);
                a.rootL[(size_t)ln.l * a.S_pad + ln.s] = Lt;
            }
            top_shift<M, T>(raw);
            ++j;
        }
        lds_barrier();
    }
    // the pattern's summed exponent: the rows' sums in row order, then the
    // clade launch's parts
    __shared__ int red[NS][TP];
    red[row][ln.ps] = esum;
    __syncthreads();
    if (row == 0) {
        int tot = 0;
        for (int i = 0; i < NS; ++i) tot += red[i][ln.ps];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < a.n_cl_esum) tot += parts[q];
        a.rootE[(size_t)ln.l * a.S_pad + ln.s] = tot;
    }
}

// q~ of internal child c: to its region slot, or to memory for a clade root
template <int M, typename T>
__device__ inline void top_store_q(const EvalArgs& a, int c, int slot, const CwLane& ln, const T qc[M], T* top) {
    if (slot) {
        T* d = top_vec<M, T>(top, slot, ln.ps);
#pragma unroll
        for (int y = 0; y < M; ++y) d[y * TP] = qc[y];
    } else {
        T* d = const_cast<T*>(node_block<M, T>(a, a.qv, c)) + ln.vec;
#pragma unroll
        for (int y = 0; y < M; ++y) d[y * TP] = qc[y];
    }
}

template <int M, typename T, bool HESS>
__device__ inline void pre_top_body(const EvalArgs& a, int tile, T* top) {
    constexpr int NS = pre_slots<T>(M);
    const int row = threadIdx.x / TP;
    const CwLane ln = top_lane<M>(a, tile);
    // the levels from the root down take this row's n nodes in decreasing
    // order: raw[k] holds node row + (n - 1 - k) NS
    static_assert(NS * TP >= 256, "one mask per thread");
    SiteVals sv;
    site_vals_load(a, ln.l, ln.s, sv);
    const unsigned long long mv = mask_load(a);
    const int n = row < a.n_sched ? min(TOP_J, (a.n_sched - 1 - row) / NS + 1) : 0;
    TopRaw<M, T> raw[TOP_J];
#pragma unroll
    for (int k = 0; k < TOP_J; ++k) top_load<M, T, false>(a, row + (n - 1 - k) * NS, ln, raw[k]);
    // rho_{s,l} gamma_l w_s from the per-category root values; the
    // category-0 tile of each pattern block also forms its logL part
    Coef cf;
    {
        SiteLik r;
        cf = site_coef(a, ln.l, ln.s, sv, r);
        if (ln.l == 0 && row == 0) logl_block_part(a, ln.pb, ln.ps, r);
    }
    __shared__ unsigned long long lmask[256];
    mask_store(lmask, mv);
    __syncthreads();
    int j = n - 1;
    for (int h = a.n_levels - 1; h >= 0; --h) {
        if (j >= 0 && row + j * NS >= uniform_int(a.level_off, h)) {
            const TopRaw<M, T>& r = raw[0];
            const int4 nd = r.nd;
            T q[M];
            if (nd.x == a.root) {
#pragma unroll
                for (int x = 0; x < M; ++x) q[x] = T(pientry<M>(a, x));
            } else {
                top_vec_load<M, T>(top, rslot(nd.w, 0), ln.ps, q);
            }
            T m0[M], m1[M], u0[M], u1[M];
            child_msg_all<M, T>(a, nd.y, r.c0, lmask, m0);
            child_msg_all<M, T>(a, nd.z, r.c1, lmask, m1);
#pragma unroll
            for (int x = 0; x < M; ++x) {
                u0[x] = q[x] * m1[x];
                u1[x] = q[x] * m0[x];
            }
            const double rden = node_rden<M, T>(u0, m0);
            double t0, t1, h0 = 0.0, h1 = 0.0;
            T q0[M], q1[M];
            const bool in0 = pre_child_core<M, T, HESS, false>(a, nd.y, ln.l, tile, ln.s, ln.ps, cf, u0, m0, rden,
                                                               r.c0.pe, t0, h0, q0);
            if constexpr (!PAIR_TERMS<HESS, false>) store_terms<HESS, T>(a, tile, ln.ps, nd.y, t0, h0);
            const bool in1 = pre_child_core<M, T, HESS, false>(a, nd.z, ln.l, tile, ln.s, ln.ps, cf, u1, m1, rden,
                                                               r.c1.pe, t1, h1, q1);
            if constexpr (!PAIR_TERMS<HESS, false>) store_terms<HESS, T>(a, tile, ln.ps, nd.z, t1, h1);
            else store_pair_terms<HESS, T>(a, tile, ln.ps, nd, t0, t1, h0, h1);
            if (in0) top_store_q<M, T>(a, nd.y, rslot(nd.w, 1), ln, q0, top);
            if (in1) top_store_q<M, T>(a, nd.z, rslot(nd.w, 2), ln, q1, top);
            top_shift<M, T>(raw);
            --j;
        }
        lds_barrier();
    }
}

// One tile per workgroup, as the level walk; two resident workgroups per CU
// hold every tile of a 500-tile launch.
template <int M, typename T>
__global__ void __launch_bounds__(post_slots<T>(M) * TP)
__attribute__((amdgpu_waves_per_eu(post_slots<T>(M) * TP / 128))) post_top_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    post_top_body<M, T>(a, blockIdx.x, reinterpret_cast<T*>(lds_dyn));
}
template <int M, typename T, bool HESS>
__global__ void __launch_bounds__(pre_slots<T>(M) * TP)
__attribute__((amdgpu_waves_per_eu(pre_slots<T>(M) * TP / 128))) pre_top_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    pre_top_body<M, T, HESS>(a, blockIdx.x, reinterpret_cast<T*>(lds_dyn));
}
template <int M, typename T>
__global__ void __launch_bounds__(post_slots<T>(M) * TP)
__attribute__((amdgpu_waves_per_eu(post_slots<T>(M) * TP / 128)))
post_top_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    post_top_body<M, T>(reqs[m.x], m.y, reinterpret_cast<T*>(lds_dyn));
}
template <int M, typename T>
__global__ void __launch_bounds__(pre_slots<T>(M) * TP)
__attribute__((amdgpu_waves_per_eu(pre_slots<T>(M) * TP / 128)))
pre_top_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    pre_top_body<M, T, false>(reqs[m.x], m.y, reinterpret_cast<T*>(lds_dyn));
}

// ---------------------------------------------------------------- gradient reduction
//
// g_b = sum over tiles of the tile sums, in a fixed order: a block owns
// GS_BRANCHES branches; its GS_SUB sub-lanes per branch sum interleaved tile
// ranges in tile order, and the GS_SUB partial sums are combined by a fixed
// binary tree.  One extra block computes logL.

constexpr int GS_THREADS = 1024;
constexpr int GS_SUB = GS_THREADS / GS_BRANCHES;

__device__ inline void gsum_body(const EvalArgs& a, int block) {
    const int nbc = gsum_blocks(a.n_branches);
    if (block == nbc) {
        finish_logl<GS_THREADS>(a);
        return;
    }
    const int B = a.n_branches;
    const int bl = threadIdx.x % GS_BRANCHES, sl = threadIdx.x / GS_BRANCHES;
    const int b = block * GS_BRANCHES + bl;
    // tile sums t = sl, sl + GS_SUB, ... added in increasing t; a chunk of
    // GS_UNROLL loads is issued before any of it is added (out-of-range
    // entries are +0.0, which leaves the sum unchanged)
    constexpr int GS_UNROLL = 8;
    double acc = 0.0;
    if (b < B) {
        const double* src = a.partial + b;
        for (int t0 = sl; t0 < a.n_tiles; t0 += GS_UNROLL * GS_SUB) {
            double v[GS_UNROLL];
#pragma unroll
            for (int j = 0; j < GS_UNROLL; ++j) {
                const int t = t0 + j * GS_SUB;
                v[j] = (t < a.n_tiles) ? src[(size_t)t * B] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < GS_UNROLL; ++j) acc += v[j];
        }
    }
    __shared__ double red[GS_SUB][GS_BRANCHES];
    red[sl][bl] = acc;
    __syncthreads();
    for (int w = GS_SUB / 2; w > 0; w >>= 1) {
        if (sl < w) red[sl][bl] += red[sl + w][bl];
        __syncthreads();
    }
    if (sl == 0 && b < B) a.grad_out[b] = red[0][bl];
}

// ---------------------------------------------------------------- entry points
//
// Each kernel has a single-evaluation entry (EvalArgs by value, block =
// blockIdx.x) and a batched entry for continuous batching: reqs[] holds the
// EvalArgs of every evaluation in the batch and map[blockIdx.x] = {request,
// block within that request}, so one launch covers all of them while each
// request keeps exactly the blocks, order and results it has alone.

template <int M, typename T>
__global__ void __launch_bounds__(256) pmat_reg_kernel(EvalArgs a) { pmat_reg_body<M, T>(a, blockIdx.x); }
template <int M, typename T>
__global__ void __launch_bounds__(256) pmat_reg_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    pmat_reg_body<M, T>(reqs[m.x], m.y);
}
template <int M, typename T>
__global__ void __launch_bounds__(256) pmat_lds_kernel(EvalArgs a) { pmat_lds_body<M, T>(a, blockIdx.x); }
template <int M, typename T>
__global__ void __launch_bounds__(256) pmat_lds_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    pmat_lds_body<M, T>(reqs[m.x], m.y);
}

template <int M, typename T>
__global__ void __launch_bounds__(post_slots<T>(M) * TP) __attribute__((amdgpu_waves_per_eu(RowMat<M>::value ? 4 : 1)))
post_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    post_body<M, T>(a, blockIdx.x, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(post_slots<T>(M) * TP) __attribute__((amdgpu_waves_per_eu(RowMat<M>::value ? 4 : 1)))
post_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    post_body<M, T>(reqs[m.x], m.y, lds_dyn);
}

template <int M, typename T, bool HESS, bool NH>
__global__ void __launch_bounds__(pre_slots<T>(M) * TP) __attribute__((amdgpu_waves_per_eu(pre_waves<T>(M))))
pre_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    pre_body<M, T, HESS, NH>(a, blockIdx.x, lds_dyn);
}
template <int M, typename T>
__global__ void __launch_bounds__(pre_slots<T>(M) * TP) __attribute__((amdgpu_waves_per_eu(pre_waves<T>(M))))
pre_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    pre_body<M, T, false, false>(reqs[m.x], m.y, lds_dyn);
}

__global__ void __launch_bounds__(GS_THREADS) gsum_kernel(EvalArgs a) { gsum_body(a, blockIdx.x); }
__global__ void __launch_bounds__(GS_THREADS) gsum_batch(const EvalArgs* __restrict__ reqs, const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    gsum_body(reqs[m.x], m.y);
}

// ---------------------------------------------------------------- dispatch

bool kernel_supported(int M, int precision) {
    if (precision == PG_SPLIT_BF16) return M >= 2 && M <= MP;
    return (M == 4 || M == 20) && (precision == PG_FP64 || precision == PG_FP32);
}

template <int M, typename T>
static hipError_t pmat_launch(const EvalArgs& a, hipStream_t st) {
    const int n = (a.blist ? a.n_blist : a.n_branches) * a.K;
    if constexpr (M <= 8) pmat_reg_kernel<M, T><<<(n + 255) / 256, 256, 0, st>>>(a);
    else pmat_lds_kernel<M, T><<<n, 256, 0, st>>>(a);
    return hipGetLastError();
}

// The small-state kernels of this file (M = 4); the dense-state path
// (kernels_dense.hip) takes 16 < M <= 32 and the split-BF16 path
// (kernels_mfma.hip) any M for PG_SPLIT_BF16.
#define PG_DISPATCH(FN, ...)                                                     \
    do {                                                                         \
        if (a.M == 4 && precision == PG_FP64) return FN<4, double>(__VA_ARGS__);   \
        if (a.M == 4 && precision == PG_FP32) return FN<4, float>(__VA_ARGS__);    \
        return hipErrorInvalidValue;                                             \
    } while (0)

hipError_t launch_pmat(const EvalArgs& a, int precision, hipStream_t st) {
    if (precision == PG_SPLIT_BF16) return launch_mfma_pmat(a, st);
    if (dense_states(a.M)) return launch_dense_pmat(a, precision, st);
    PG_DISPATCH(pmat_launch, a, st);
}

// Clade walks in their own launches (when the context has the exponent
// buffer they need): the arguments of the top-level launch drop the clades.
size_t cw_lds_bytes(const EvalArgs& a, size_t elem) {
    return elem * (size_t)CW_WAVES * CW_ROWS * a.cl_depth * a.M * TP;
}
int cw_groups(const EvalArgs& a) { return (a.n_tiles + CW_ROWS - 1) / CW_ROWS; }
static bool split_clades(const EvalArgs& a) {
    // the separate walks form element offsets in 32 bits
    const size_t vec_elems = (size_t)a.n_nodes * a.n_tiles * a.M * TP;
    return a.n_cl > 0 && a.cl_esum != nullptr && vec_elems < (size_t(1) << 31) &&
           (size_t)a.n_nodes * a.S_pad < (size_t(1) << 31);
}
static EvalArgs top_only(const EvalArgs& a, int n_esum) {
    EvalArgs t = a;
    t.n_cl = 0;
    t.cl_depth = 0;
    t.n_cl_esum = n_esum;
    return t;
}
static bool small_clades(const EvalArgs& a, int precision) {
    return (precision == PG_FP64 || precision == PG_FP32) && a.M * a.M <= TP && split_clades(a);
}
static int clade_parts(int precision) {
    return (precision == PG_FP32 ? post_slots<float>(4) : post_slots<double>(4)) / CW_WAVES;
}
int clade_blocks(const EvalArgs& a, int precision) {
    return small_clades(a, precision) ? cw_groups(a) * clade_parts(precision) : 0;
}
EvalArgs clade_top_args(const EvalArgs& a, int precision) {
    return small_clades(a, precision) ? top_only(a, clade_parts(precision)) : a;
}
size_t clade_lds_bytes(const EvalArgs& a, int precision) {
    return small_clades(a, precision) ? cw_lds_bytes(a, precision == PG_FP32 ? 4 : 8) : 0;
}

// The top levels take the prefetching launches when they are one region
// (every top level narrow enough, at most TOP_J nodes per row) and no
// per-node exponents of partial re-evaluation are kept.
static bool top_prefetch(const EvalArgs& t, int ns) {
    return t.n_cl == 0 && t.top_level == 0 && t.n_sched >= 1 && t.top_nodes == t.n_sched &&
           t.n_sched <= TOP_J * ns && t.expo == nullptr && !t.expo_delta;
}

// Whether a request's top-level launch arguments (clade_top_args) take the
// top-level launches above in a batch, and their dynamic LDS.
bool top_launch_ok(const EvalArgs& t, int precision) {
    if (!(t.M == 4 && (precision == PG_FP64 || precision == PG_FP32))) return false;
    const int ns = precision == PG_FP32 ? post_slots<float>(4) : post_slots<double>(4);
    return top_prefetch(t, ns) && t.n_cl_esum >= 1 && t.n_cl_esum <= ns / CW_WAVES && t.n_models == 0;
}
size_t top_launch_lds(const EvalArgs& t, int precision) { return top_lds_bytes(t, precision == PG_FP32 ? 4 : 8); }

template <int M, typename T>
static hipError_t post_launch(const EvalArgs& a, hipStream_t st) {
    const int prec = sizeof(T) == 4 ? PG_FP32 : PG_FP64;
    if (a.n_cl > 0 && !(RowMat<M>::value && split_clades(a))) return hipErrorInvalidValue;
    if (a.n_cl > 0) {
        constexpr int NQ = post_slots<T>(M) / CW_WAVES;
        post_clade_kernel<M, T><<<cw_groups(a) * NQ, CW_WAVES * 64, cw_lds_bytes(a, sizeof(T)), st>>>(a);
        const EvalArgs t = top_only(a, NQ);
        if (top_prefetch(t, post_slots<T>(M)) && t.n_cl_esum >= 1 && t.n_cl_esum <= NQ)
            post_top_kernel<M, T><<<a.n_tiles, post_slots<T>(M) * TP, top_lds_bytes(t, sizeof(T)), st>>>(t);
        else
            post_kernel<M, T><<<a.n_tiles, post_slots<T>(M) * TP, post_lds_bytes(t, prec), st>>>(t);
        return hipGetLastError();
    }
    post_kernel<M, T><<<a.n_tiles, post_slots<T>(M) * TP, post_lds_bytes(a, prec), st>>>(a);
    return hipGetLastError();
}

hipError_t launch_post(const EvalArgs& a, int precision, hipStream_t st) {
    if (precision == PG_SPLIT_BF16) return launch_mfma_post(a, st);
    if (dense_states(a.M)) return launch_dense_post(a, precision, st);
    PG_DISPATCH(post_launch, a, st);
}

hipError_t launch_logl(const EvalArgs& a, hipStream_t st) {
    logl_kernel<<<1, LOGL_THREADS, 0, st>>>(a);
    return hipGetLastError();
}

template <int M, typename T, bool HESS, bool NH>
static void pre_launch_variant(const EvalArgs& a, hipStream_t st) {
    const int prec = sizeof(T) == 4 ? PG_FP32 : PG_FP64;
    const dim3 block(pre_slots<T>(M) * TP);
    if (a.n_cl > 0) {
        constexpr int NQ = pre_slots<T>(M) / CW_WAVES;
        const EvalArgs t = top_only(a, 0);
        if (!NH && top_prefetch(t, pre_slots<T>(M)))
            pre_top_kernel<M, T, HESS><<<a.n_tiles, block, top_lds_bytes(t, sizeof(T)), st>>>(t);
        else
            pre_kernel<M, T, HESS, NH><<<a.n_tiles, block, pre_lds_bytes(t, prec), st>>>(t);
        pre_clade_kernel<M, T, HESS, NH><<<cw_groups(a) * NQ, CW_WAVES * 64, cw_lds_bytes(a, sizeof(T)), st>>>(a);
        return;
    }
    pre_kernel<M, T, HESS, NH><<<a.n_tiles, block, pre_lds_bytes(a, prec), st>>>(a);
}

template <int M, typename T>
static hipError_t pre_launch(const EvalArgs& a, hipStream_t st, bool hess) {
    if (a.n_cl > 0 && !(RowMat<M>::value && split_clades(a))) return hipErrorInvalidValue;
    if (a.n_models) {
        if (hess) pre_launch_variant<M, T, true, true>(a, st);
        else pre_launch_variant<M, T, false, true>(a, st);
    } else {
        if (hess) pre_launch_variant<M, T, true, false>(a, st);
        else pre_launch_variant<M, T, false, false>(a, st);
    }
    return hipGetLastError();
}

hipError_t launch_pre(const EvalArgs& a, int precision, hipStream_t st, bool hess) {
    if (precision == PG_SPLIT_BF16) return launch_mfma_pre(a, st, hess);
    if (dense_states(a.M)) return launch_dense_pre(a, precision, st, hess);
    PG_DISPATCH(pre_launch, a, st, hess);
}

// ---------------------------------------------------------------- Hessian reduction
//
// One block per branch b:
//   d2 logL/dt_b^2 = sum_t partial2[t][b] - sum_s w_s (sum_l r1[b][l][s])^2,
// both sums in a fixed order (strided per thread, then a fixed tree).
constexpr int HS_THREADS = 256;

__global__ void __launch_bounds__(HS_THREADS) hsum_kernel(EvalArgs a) {
    const int b = blockIdx.x;
    const int B = a.n_branches;
    double sq = 0.0, p2 = 0.0;
    for (int s = threadIdx.x; s < a.S_pad; s += HS_THREADS) {
        double g = 0.0;
        for (int l = 0; l < a.K; ++l) g += a.r1[((size_t)b * a.K + l) * a.S_pad + s];
        sq += a.weights[s] * g * g;
    }
    for (int t = threadIdx.x; t < a.n_tiles; t += HS_THREADS) p2 += a.partial2[(size_t)t * B + b];
    __shared__ double rs[HS_THREADS], rp[HS_THREADS];
    rs[threadIdx.x] = sq;
    rp[threadIdx.x] = p2;
    __syncthreads();
    for (int w = HS_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            rp[threadIdx.x] += rp[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.hess_out[b] = rp[0] - rs[0];
}

hipError_t launch_hsum(const EvalArgs& a, hipStream_t st) {
    hsum_kernel<<<a.n_branches, HS_THREADS, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_gsum(const EvalArgs& a, hipStream_t st) {
    gsum_kernel<<<gsum_blocks(a.n_branches) + 1, GS_THREADS, 0, st>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- batched launches

int pmat_blocks(const EvalArgs& a, int precision) {
    return (a.M <= 8 && precision != PG_SPLIT_BF16) ? (a.n_branches * a.K + 255) / 256 : a.n_branches * a.K;
}
int traversal_blocks(const EvalArgs& a) { return a.n_tiles; }
int gsum_total_blocks(const EvalArgs& a) { return gsum_blocks(a.n_branches) + 1; }

size_t post_lds_bytes(const EvalArgs& a, int precision) {
    if (precision == PG_SPLIT_BF16) return mfma_post_lds_bytes(a);
    return sched_lds_bytes(a);
}
size_t pre_lds_bytes(const EvalArgs& a, int precision) {
    if (precision == PG_SPLIT_BF16) return mfma_pre_lds_bytes(a);
    const size_t es = precision == PG_FP32 ? 4 : 8;
    return sched_lds_bytes(a) + top_lds_bytes(a, es);
}

template <int M, typename T>
static hipError_t batch_launch(const BatchLaunch& b, hipStream_t st) {
    if (b.pmat_blocks > 0) {
        if constexpr (M <= 8) pmat_reg_batch<M, T><<<b.pmat_blocks, 256, 0, st>>>(b.reqs, b.pmat_map);
        else pmat_lds_batch<M, T><<<b.pmat_blocks, 256, 0, st>>>(b.reqs, b.pmat_map);
    }
    // requests with clades: their clade walks in the clade launches, their
    // top levels in the traversal launches (reqs_top)
    const EvalArgs* top = b.reqs_top ? b.reqs_top : b.reqs;
    if (b.clade_blocks > 0)
        post_clade_batch<M, T><<<b.clade_blocks, CW_WAVES * 64, b.clade_lds, st>>>(b.reqs, b.clade_map);
    if (b.top_kernels) {
        post_top_batch<M, T><<<b.trav_blocks, post_slots<T>(M) * TP, b.top_lds, st>>>(top, b.trav_map);
        pre_top_batch<M, T><<<b.trav_blocks, pre_slots<T>(M) * TP, b.top_lds, st>>>(top, b.trav_map);
    } else {
        post_batch<M, T><<<b.trav_blocks, post_slots<T>(M) * TP, b.post_lds, st>>>(top, b.trav_map);
        pre_batch<M, T><<<b.trav_blocks, pre_slots<T>(M) * TP, b.pre_lds, st>>>(top, b.trav_map);
    }
    if (b.clade_blocks > 0)
        pre_clade_batch<M, T><<<b.clade_blocks, CW_WAVES * 64, b.clade_lds, st>>>(b.reqs, b.clade_map);
    gsum_batch<<<b.gsum_blocks, GS_THREADS, 0, st>>>(b.reqs, b.gsum_map);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchLaunch& b, hipStream_t st) {
    const int M = b.M, precision = b.precision;
    if (precision == PG_SPLIT_BF16) {
        const hipError_t e = launch_mfma_batch(b, st);
        if (e != hipSuccess) return e;
        gsum_batch<<<b.gsum_blocks, GS_THREADS, 0, st>>>(b.reqs, b.gsum_map);
        return hipGetLastError();
    }
    if (M == 4 && precision == PG_FP64) return batch_launch<4, double>(b, st);
    if (M == 4 && precision == PG_FP32) return batch_launch<4, float>(b, st);
    if (dense_states(M)) {
        const hipError_t e = launch_dense_batch(b, st);
        if (e != hipSuccess) return e;
        gsum_batch<<<b.gsum_blocks, GS_THREADS, 0, st>>>(b.reqs, b.gsum_map);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace pg
