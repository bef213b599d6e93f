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
__device__ __attribute__((always_inline)) inline bool taylor_F_lds(const EvalArgs& a, int b, int l, double* A,
                                                                   double* G, double* W) {
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

// F = P - I of branch b, category l from the eigen-decomposition Q =
// V B V^-1 (a.eV, a.eVinv: M x M row-major; B block diagonal, a.eKind[j] 0
// for a real eigenvalue a.eRe[j], 1 / 2 for the two columns of a conjugate
// pair a.eRe[j] +- i a.eIm[j]):
//   F = V X,  X = (exp(B tau) - I) V^-1,  tau = rate_l t_b,
// where row j of X is C_j r_j (real eigenvalue, C = expm1(re tau)) or, for a
// pair j, j+1 with a = re tau, w = im tau, C = e^a cos w - 1 and
// S = e^a sin w: C r_j + S r_{j+1} and -S r_j + C r_{j+1} (r_j: row j of
// V^-1).  Left in W; V and X are staged in A and G, fc / fs hold M
// coefficients.  Returns false when t_b is not finite and >= 0.
template <int M>
__device__ __attribute__((always_inline)) inline bool eigen_F_lds(const EvalArgs& a, int b, int l, double* A,
                                                                  double* G, double* W, double* fc, double* fs) {
    const double tb = a.t[b];
    if (bad_length(tb)) return false;
    const double tau = a.rates[l] * tb;
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const int kind = a.eKind[j];
        const double ar = a.eRe[j] * tau;
        double C, S = 0.0;
        if (kind == 0) {
            C = expm1(ar);
        } else {
            const double wi = a.eIm[j] * tau;
            const double sh = sin(0.5 * wi);
            C = expm1(ar) * cos(wi) - 2.0 * sh * sh;  // e^a cos w - 1
            S = exp(ar) * sin(wi);
        }
        fc[j] = C;
        fs[j] = kind == 1 ? S : kind == 2 ? -S : 0.0;  // coefficient of the partner row
    }
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        A[e] = a.eV[e];
        G[e] = a.eVinv[e];
    }
    __syncthreads();
    // X = (exp(B tau) - I) V^-1 in W, then F = V X in G
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        const int j = e / M, y = e % M;
        const int kind = a.eKind[j];
        const int partner = kind == 1 ? j + 1 : kind == 2 ? j - 1 : j;
        W[e] = fc[j] * G[e] + fs[j] * G[partner * M + y];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
        const int i = e / M, y = e % M;
        double acc = 0.0;
        for (int j = 0; j < M; ++j) acc = fma(A[i * M + j], W[j * M + y], acc);
        G[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) W[e] = G[e];
    __syncthreads();
    return true;
}

}  // namespace pg
