// Transition matrices P = exp(Q_b rate_l t_b) in FP64 for one (branch,
// category) per workgroup, by scaling and squaring of the Taylor series,
// carried in the form P = I + F so the small off-diagonal entries and the
// 1 - small diagonal keep full relative accuracy:
//   scale A = Q_b rate_l t_b by 2^-s so that ||A||_inf <= 1/2,
//   F = A (I + A/2 (I + A/3 (... (I + A/DEG)))),      truncation < 1e-19,
//   s times: F <- 2F + F F   ((I+F)^2 = I + 2F + F^2),
//   P = I + F.
// A branch length that is negative or not finite gives no matrix (the
// callers write NaN, which propagates to a NaN logL).
#pragma once

#include "pg_internal.h"

namespace pg {

constexpr int TAYLOR_DEG = 16;

// Rate matrix and its norm on branch b: the model's, or the branch's own
// in a non-homogeneous model.
__device__ inline const double* branch_q(const EvalArgs& a, int b, int M) {
    return a.n_models ? a.Qm + (size_t)a.branch_model[b] * M * M : a.Q64;
}
__device__ inline double branch_qnorm(const EvalArgs& a, int b) {
    return a.n_models ? a.qnorm_m[a.branch_model[b]] : a.qnorm;
}

__device__ inline bool bad_length(double t) { return !(t >= 0.0) || isinf(t); }

// F = P - I of branch b, category l, left in W (M x M row-major in LDS; A
// and G are LDS scratch of the same size).  The whole workgroup calls it;
// returns false (and leaves W undefined) when t_b is not finite and >= 0.
template <int M>
__device__ inline bool taylor_F_lds(const EvalArgs& a, int b, int l, double* A, double* G, double* W) {
    const double tb = a.t[b];
    if (bad_length(tb)) return false;
    const double h = a.rates[l] * tb;
    const double* Qb = branch_q(a, b, M);
    double nrm = branch_qnorm(a, b) * h;
    int s = 0;
    while (nrm > 0.5 && s < 1100) { nrm *= 0.5; ++s; }
    const double hs = ldexp(h, -s);
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        A[e] = Qb[e] * hs;
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
    return true;
}

}  // namespace pg
