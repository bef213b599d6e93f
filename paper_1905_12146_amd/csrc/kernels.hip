// Device kernels of one evaluation: transition matrices, post-order pass,
// root integration, pre-order pass fused with the gradient, and the
// fixed-order reduction of per-tile gradient sums.
//
// Data layout in HBM (pattern index fastest, so a group of 16 lanes that
// handles 16 consecutive patterns reads one contiguous run per state):
//   P     [branch][category][x][y]       x = parent state, y = child state
//   msg   [internal node - N][category][state][pattern]   message P_k p~_k
//   qv    [internal node - N][category][state][pattern]   pre-order q~_k
//   codes [tip][pattern]                 uint8 code of the tip observation
//
// Work decomposition: a workgroup owns one tile = 16 consecutive patterns
// of one rate category and walks the whole tree for it, level by level
// (nodes of equal height are independent).  Its 256 threads are 16 node
// slots x 16 pattern lanes; a barrier separates levels.  Tiles never
// communicate, so there is no grid-wide synchronisation inside a pass.
//
// Rescaling is per node, per pattern and per category, by an exact power of
// two.  Categories therefore never mix inside the traversal: the per-site
// likelihood L_s = sum_l w_l L_{s,l} is formed once at the root from each
// category's scaled value and summed exponent, and the gradient uses
//   d log L_s / dt_b = sum_l rho_{s,l} gamma_l (u^T Q m)/(u^T m),
//   rho_{s,l} = w_l L_{s,l} / L_s,
// which equals Eq. (GradientWithGamma) of Section 2.6 (u^T m = L_{s,l} up to
// the category's own scale factor, which cancels in each ratio).
#include "pg_internal.h"

#include <climits>

namespace pg {

// ---------------------------------------------------------------- helpers

__device__ inline int exp_of(double x) { int e; (void)frexp(x, &e); return e; }
__device__ inline int exp_of(float x) { int e; (void)frexpf(x, &e); return e; }
__device__ inline double pow2_scale(double x, int e) { return ldexp(x, e); }
__device__ inline float pow2_scale(float x, int e) { return ldexpf(x, e); }

// Sum over the 16 lanes of a node slot; every lane gets the same value.
__device__ inline double sum16(double v) {
    v += __shfl_xor(v, 1, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 8, 16);
    return v;
}

// Outgoing message of child c for category l and pattern s: the stored
// P_c p~_c for an internal child, P_c times the tip indicator for a tip
// (a column of P_c, or the sum of the allowed columns).
template <int M, typename T>
__device__ inline void child_message(const EvalArgs& a, int c, int l, int s, T out[M]) {
    const T* P = static_cast<const T*>(a.P);
    if (c < a.n_tips) {
        const T* Pc = P + ((size_t)c * a.K + l) * M * M;
        const unsigned code = a.codes[(size_t)c * a.S_pad + s];
        if (code < (unsigned)M) {
#pragma unroll
            for (int x = 0; x < M; ++x) out[x] = Pc[x * M + code];
        } else {
            const unsigned long long mask = a.masks[code];
#pragma unroll
            for (int x = 0; x < M; ++x) {
                T acc = T(0);
#pragma unroll
                for (int y = 0; y < M; ++y)
                    if ((mask >> y) & 1ull) acc += Pc[x * M + y];
                out[x] = acc;
            }
        }
    } else {
        const T* src = static_cast<const T*>(a.msg) +
                       ((size_t)(c - a.n_tips) * a.K + l) * M * a.S_pad + s;
#pragma unroll
        for (int x = 0; x < M; ++x) out[x] = src[(size_t)x * a.S_pad];
    }
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

constexpr int TAYLOR_DEG = 16;

__device__ inline bool bad_length(double t) { return !(t >= 0.0) || isinf(t); }

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
__global__ void __launch_bounds__(256) pmat_reg_kernel(EvalArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n_branches * a.K) return;
    const int b = idx / a.K, l = idx % a.K;
    double tb = a.t[b];
    if (bad_length(tb)) {
        atomicOr(a.status, 1);
        tb = 0.0;
    }
    const double h = a.rates[l] * tb;
    double nrm = a.qnorm * h;
    int s = 0;
    while (nrm > 0.5 && s < 1100) { nrm *= 0.5; ++s; }
    const double hs = ldexp(h, -s);
    double A[M][M], G[M][M], W[M][M];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) {
            A[i][j] = a.Q64[i * M + j] * hs;
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
    T* out = static_cast<T*>(a.P) + ((size_t)b * a.K + l) * M * M;
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
        for (int j = 0; j < M; ++j) out[i * M + j] = T(((i == j) ? 1.0 : 0.0) + W[i][j]);
}

// One workgroup per (branch, category); matrices in LDS (larger M).
template <int M, typename T>
__global__ void __launch_bounds__(256) pmat_lds_kernel(EvalArgs a) {
    __shared__ double A[M * M], G[M * M], W[M * M];
    const int idx = blockIdx.x;
    const int b = idx / a.K, l = idx % a.K;
    double tb = a.t[b];
    if (bad_length(tb)) {
        if (threadIdx.x == 0) atomicOr(a.status, 1);
        tb = 0.0;
    }
    const double h = a.rates[l] * tb;
    double nrm = a.qnorm * h;
    int s = 0;
    while (nrm > 0.5 && s < 1100) { nrm *= 0.5; ++s; }
    const double hs = ldexp(h, -s);
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        A[e] = a.Q64[e] * hs;
        G[e] = (e / M == e % M) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = TAYLOR_DEG; k >= 2; --k) {
        const double inv = 1.0 / k;
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
            const int i = e / M, j = e % M;
            double acc = 0.0;
            for (int q = 0; q < M; ++q) acc = fma(A[i * M + q], G[q * M + j], acc);
            W[e] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < M * M; e += blockDim.x)
            G[e] = ((e / M == e % M) ? 1.0 : 0.0) + W[e] * inv;
        __syncthreads();
    }
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        const int i = e / M, j = e % M;
        double acc = 0.0;
        for (int q = 0; q < M; ++q) acc = fma(A[i * M + q], G[q * M + j], acc);
        W[e] = acc;
    }
    __syncthreads();
    for (int r = 0; r < s; ++r) {
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
            const int i = e / M, j = e % M;
            double acc = 0.0;
            for (int q = 0; q < M; ++q) acc = fma(W[i * M + q], W[q * M + j], acc);
            G[e] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) W[e] = 2.0 * W[e] + G[e];
        __syncthreads();
    }
    T* out = static_cast<T*>(a.P) + ((size_t)b * a.K + l) * M * M;
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

template <int M, typename T>
__global__ void __launch_bounds__(WG) post_kernel(EvalArgs a) {
    const int tile = blockIdx.x;
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int ps = threadIdx.x % TP, ns = threadIdx.x / TP;
    const int s = pb * TP + ps;
    const T* P = static_cast<const T*>(a.P);
    T* msg = static_cast<T*>(a.msg);
    int esum = 0;
    for (int h = 0; h < a.n_levels; ++h) {
        const int beg = a.level_off[h], end = a.level_off[h + 1];
        for (int idx = beg + ns; idx < end; idx += NS) {
            const int k = a.level_nodes[idx];
            const int2 ch = a.children[k];
            T mi[M], mj[M], p[M];
            child_message<M, T>(a, ch.x, l, s, mi);
            child_message<M, T>(a, ch.y, l, s, mj);
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
            esum += e;
            if (k != a.root) {
                const T* Pk = P + ((size_t)k * a.K + l) * M * M;
                T* out = msg + ((size_t)(k - a.n_tips) * a.K + l) * M * a.S_pad + s;
#pragma unroll
                for (int x = 0; x < M; ++x) {
                    T acc = T(0);
#pragma unroll
                    for (int y = 0; y < M; ++y) acc = fma(Pk[x * M + y], p[y], acc);
                    out[(size_t)x * a.S_pad] = acc;
                }
            } else {
                double Lt = 0.0;
#pragma unroll
                for (int x = 0; x < M; ++x) Lt = fma(a.pi64[x], (double)p[x], Lt);
                a.rootL[(size_t)l * a.S_pad + s] = Lt;
            }
        }
        __syncthreads();
    }
    __shared__ int red[NS][TP];
    red[ns][ps] = esum;
    __syncthreads();
    if (ns == 0) {
        int tot = 0;
        for (int i = 0; i < NS; ++i) tot += red[i][ps];
        a.rootE[(size_t)l * a.S_pad + s] = tot;
    }
}

// ---------------------------------------------------------------- root
//
// L_s = sum_l w_l L~_{s,l} 2^{E_{s,l}}  (Eq. discreteRateLikelihood), formed
// relative to the largest exponent so nothing under- or overflows;
// rho_{s,l} = w_l L_{s,l} / L_s; logL = sum_s w_s log L_s.  One workgroup,
// fixed-order reduction.

constexpr int ROOT_THREADS = 1024;

__global__ void __launch_bounds__(ROOT_THREADS) root_kernel(EvalArgs a) {
    const double LN2 = 0.69314718055994530942;
    double acc = 0.0;
    int zero = 0;
    for (int s = threadIdx.x; s < a.S_pad; s += ROOT_THREADS) {
        int emax = INT_MIN;
        for (int l = 0; l < a.K; ++l)
            if (a.rootL[(size_t)l * a.S_pad + s] > 0.0) emax = max(emax, a.rootE[(size_t)l * a.S_pad + s]);
        double tot = 0.0;
        if (emax != INT_MIN)
            for (int l = 0; l < a.K; ++l) {
                const double L = a.rootL[(size_t)l * a.S_pad + s];
                if (L > 0.0) tot += a.catw[l] * ldexp(L, a.rootE[(size_t)l * a.S_pad + s] - emax);
            }
        const double w = a.weights[s];
        if (tot > 0.0) {
            for (int l = 0; l < a.K; ++l) {
                const double L = a.rootL[(size_t)l * a.S_pad + s];
                a.rho[(size_t)l * a.S_pad + s] =
                    (L > 0.0) ? a.catw[l] * ldexp(L, a.rootE[(size_t)l * a.S_pad + s] - emax) / tot : 0.0;
            }
            if (w > 0.0) acc += w * (log(tot) + (double)emax * LN2);
        } else {
            for (int l = 0; l < a.K; ++l) a.rho[(size_t)l * a.S_pad + s] = 0.0;
            if (w > 0.0) zero = 1;
        }
    }
    __shared__ double red[ROOT_THREADS];
    __shared__ int zred[ROOT_THREADS];
    red[threadIdx.x] = acc;
    zred[threadIdx.x] = zero;
    __syncthreads();
    for (int w = ROOT_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] += red[threadIdx.x + w];
            zred[threadIdx.x] |= zred[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (zred[0]) {
            atomicOr(a.status, 2);
            a.logL[0] = -INFINITY;
        } else {
            a.logL[0] = red[0];
        }
    }
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

template <int M, typename T>
__device__ inline void pre_child(const EvalArgs& a, int c, int l, int s, int tile, int ps, double coef,
                                 const T q[M], const T msib[M], const T mown[M]) {
    T u[M];
#pragma unroll
    for (int x = 0; x < M; ++x) u[x] = q[x] * msib[x];
    T den = T(0), num = T(0);
#pragma unroll
    for (int x = 0; x < M; ++x) {
        T qm = T(0);
#pragma unroll
        for (int y = 0; y < M; ++y) qm = fma(T(a.Q64[x * M + y]), mown[y], qm);
        num = fma(u[x], qm, num);
        den = fma(u[x], mown[x], den);
    }
    double term = (coef > 0.0 && den > T(0)) ? coef * ((double)num / (double)den) : 0.0;
    term = sum16(term);
    if (ps == 0) a.partial[(size_t)tile * a.n_branches + c] = term;
    if (c >= a.n_tips) {
        const T* Pc = static_cast<const T*>(a.P) + ((size_t)c * a.K + l) * M * M;
        T qc[M];
        T mx = T(0);
#pragma unroll
        for (int y = 0; y < M; ++y) {
            T acc = T(0);
#pragma unroll
            for (int x = 0; x < M; ++x) acc = fma(Pc[x * M + y], u[x], acc);
            qc[y] = acc;
            mx = fmax(mx, acc);
        }
        const int e = (mx > T(0)) ? exp_of(mx) : 0;
        T* out = static_cast<T*>(a.qv) + ((size_t)(c - a.n_tips) * a.K + l) * M * a.S_pad + s;
#pragma unroll
        for (int y = 0; y < M; ++y) out[(size_t)y * a.S_pad] = pow2_scale(qc[y], -e);
    }
}

template <int M, typename T>
__global__ void __launch_bounds__(WG) pre_kernel(EvalArgs a) {
    const int tile = blockIdx.x;
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int ps = threadIdx.x % TP, ns = threadIdx.x / TP;
    const int s = pb * TP + ps;
    const double coef = a.weights[s] * a.rho[(size_t)l * a.S_pad + s] * a.rates[l];
    for (int h = a.n_levels - 1; h >= 0; --h) {
        const int beg = a.level_off[h], end = a.level_off[h + 1];
        for (int idx = beg + ns; idx < end; idx += NS) {
            const int k = a.level_nodes[idx];
            const int2 ch = a.children[k];
            T q[M], mi[M], mj[M];
            if (k == a.root) {
#pragma unroll
                for (int x = 0; x < M; ++x) q[x] = T(a.pi64[x]);
            } else {
                const T* src = static_cast<const T*>(a.qv) +
                               ((size_t)(k - a.n_tips) * a.K + l) * M * a.S_pad + s;
#pragma unroll
                for (int x = 0; x < M; ++x) q[x] = src[(size_t)x * a.S_pad];
            }
            child_message<M, T>(a, ch.x, l, s, mi);
            child_message<M, T>(a, ch.y, l, s, mj);
            pre_child<M, T>(a, ch.x, l, s, tile, ps, coef, q, mj, mi);
            pre_child<M, T>(a, ch.y, l, s, tile, ps, coef, q, mi, mj);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- gradient reduction
//
// g_b = sum over tiles of the tile sums, in tile order (deterministic).

__global__ void __launch_bounds__(256) gsum_kernel(EvalArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.n_branches) return;
    double acc = 0.0;
    for (int t = 0; t < a.n_tiles; ++t) acc += a.partial[(size_t)t * a.n_branches + b];
    a.grad[b] = acc;
}

// ---------------------------------------------------------------- dispatch

bool kernel_supported(int M, int precision) {
    return (M == 4 || M == 20) && (precision == PG_FP64 || precision == PG_FP32);
}

template <int M, typename T>
static hipError_t pmat_launch(const EvalArgs& a, hipStream_t st) {
    if constexpr (M <= 8) {
        const int n = a.n_branches * a.K;
        pmat_reg_kernel<M, T><<<(n + 255) / 256, 256, 0, st>>>(a);
    } else {
        pmat_lds_kernel<M, T><<<a.n_branches * a.K, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}

#define PG_DISPATCH(FN, ...)                                                   \
    do {                                                                       \
        if (a.M == 4 && precision == PG_FP64) return FN<4, double>(__VA_ARGS__); \
        if (a.M == 4 && precision == PG_FP32) return FN<4, float>(__VA_ARGS__);  \
        if (a.M == 20 && precision == PG_FP64) return FN<20, double>(__VA_ARGS__); \
        if (a.M == 20 && precision == PG_FP32) return FN<20, float>(__VA_ARGS__);  \
        return hipErrorInvalidValue;                                           \
    } while (0)

hipError_t launch_pmat(const EvalArgs& a, int precision, hipStream_t st) {
    PG_DISPATCH(pmat_launch, a, st);
}

template <int M, typename T>
static hipError_t post_launch(const EvalArgs& a, hipStream_t st) {
    post_kernel<M, T><<<a.n_tiles, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_post(const EvalArgs& a, int precision, hipStream_t st) {
    PG_DISPATCH(post_launch, a, st);
}

hipError_t launch_root(const EvalArgs& a, hipStream_t st) {
    root_kernel<<<1, ROOT_THREADS, 0, st>>>(a);
    return hipGetLastError();
}

template <int M, typename T>
static hipError_t pre_launch(const EvalArgs& a, hipStream_t st) {
    pre_kernel<M, T><<<a.n_tiles, WG, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_pre(const EvalArgs& a, int precision, hipStream_t st) {
    PG_DISPATCH(pre_launch, a, st);
}

hipError_t launch_gsum(const EvalArgs& a, hipStream_t st) {
    gsum_kernel<<<(a.n_branches + 255) / 256, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_hess(const EvalArgs&, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_hsum(const EvalArgs&, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace pg
