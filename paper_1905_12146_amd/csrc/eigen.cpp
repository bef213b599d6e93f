// Eigen-decomposition of a real rate matrix, used by the split-BF16 path to
// form transition matrices with one matrix product per branch and category:
//   Q = V B V^-1,  B block diagonal: 1x1 blocks for real eigenvalues and
//   2x2 blocks [[a, b], [-b, a]] for conjugate pairs a +- ib, whose columns
//   in V are the real and imaginary parts of the eigenvector of a + ib, so
//   exp(Q tau) - I = V (exp(B tau) - I) V^-1.
// Steps (host, FP64):
//   1. Householder reduction of Q to upper Hessenberg form;
//   2. shifted QR iterations on the Hessenberg matrix in complex arithmetic
//      (Wilkinson shifts, an exceptional shift every tenth iteration,
//      deflation at negligible subdiagonal entries) for the eigenvalues;
//   3. eigenvalues whose imaginary part is negligible are made real, the
//      others are matched into conjugate pairs;
//   4. each eigenvector by inverse iteration on Q - sigma I (LU with partial
//      pivoting), orthogonalised against earlier vectors of the same cluster
//      of nearly equal eigenvalues;
//   5. V^-1 by LU with partial pivoting, cond_1(V), and the reconstruction
//      error max |V B V^-1 - Q| / max |Q|.
// A non-diagonalisable or badly conditioned Q is reported through `ok` and
// the caller then uses scaling and squaring instead.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "pg_internal.h"

namespace pg {

namespace {

using cd = std::complex<double>;

double norm_inf(const std::vector<double>& A, int n) {
    double r = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += std::fabs(A[i * n + j]);
        r = std::max(r, s);
    }
    return r;
}

// Upper Hessenberg form of A (n x n, row-major) by Householder reflections.
void hessenberg(std::vector<double>& A, int n) {
    std::vector<double> v(n);
    for (int k = 0; k + 2 < n; ++k) {
        double nx = 0.0;
        for (int i = k + 1; i < n; ++i) nx += A[i * n + k] * A[i * n + k];
        nx = std::sqrt(nx);
        if (nx == 0.0) continue;
        const double x0 = A[(k + 1) * n + k];
        const double alpha = x0 >= 0.0 ? -nx : nx;
        double nv = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = A[i * n + k] - (i == k + 1 ? alpha : 0.0);
            nv += v[i] * v[i];
        }
        nv = std::sqrt(nv);
        if (nv == 0.0) continue;
        for (int i = k + 1; i < n; ++i) v[i] /= nv;
        // A <- (I - 2 v v^T) A
        for (int j = 0; j < n; ++j) {
            double d = 0.0;
            for (int i = k + 1; i < n; ++i) d += v[i] * A[i * n + j];
            for (int i = k + 1; i < n; ++i) A[i * n + j] -= 2.0 * v[i] * d;
        }
        // A <- A (I - 2 v v^T)
        for (int i = 0; i < n; ++i) {
            double d = 0.0;
            for (int j = k + 1; j < n; ++j) d += A[i * n + j] * v[j];
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= 2.0 * d * v[j];
        }
        for (int i = k + 2; i < n; ++i) A[i * n + k] = 0.0;
    }
}

// Eigenvalues of an upper Hessenberg matrix by shifted complex QR.
bool hessenberg_eigenvalues(const std::vector<double>& Hr, int n, std::vector<cd>& out) {
    std::vector<cd> H(Hr.begin(), Hr.end());
    auto h = [&](int i, int j) -> cd& { return H[(size_t)i * n + j]; };
    const double eps = 2.220446049250313e-16;
    double scale = 0.0;
    for (double x : Hr) scale = std::max(scale, std::fabs(x));
    if (scale == 0.0) scale = 1.0;
    out.clear();
    int hi = n - 1, iter = 0, total = 0;
    std::vector<cd> cs(n), sn(n);
    while (hi >= 0) {
        int l = hi;
        while (l > 0) {
            double s = std::abs(h(l - 1, l - 1)) + std::abs(h(l, l));
            if (s == 0.0) s = scale;
            if (std::abs(h(l, l - 1)) <= eps * s) {
                h(l, l - 1) = 0.0;
                break;
            }
            --l;
        }
        if (l == hi) {
            out.push_back(h(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 60 * n) return false;
        ++iter;
        cd mu;
        if (iter % 10 == 0) {
            mu = h(hi, hi) + cd(0.75 * std::abs(h(hi, hi - 1)), 0.25 * std::abs(h(hi, hi - 1)));
        } else {
            const cd a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        for (int k = l; k <= hi; ++k) h(k, k) -= mu;
        // H - mu I = Q R by Givens rotations G_k = [[conj c, conj s], [-s, c]]
        for (int k = l; k < hi; ++k) {
            const cd a = h(k, k), b = h(k + 1, k);
            const double r = std::hypot(std::abs(a), std::abs(b));
            cd c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = a / r;
                s = b / r;
            }
            cs[k] = c;
            sn[k] = s;
            for (int j = k; j <= hi; ++j) {
                const cd x = h(k, j), y = h(k + 1, j);
                h(k, j) = std::conj(c) * x + std::conj(s) * y;
                h(k + 1, j) = -s * x + c * y;
            }
        }
        // R Q: apply G_k^H = [[c, -conj s], [s, conj c]] on the right
        for (int k = l; k < hi; ++k) {
            const cd c = cs[k], s = sn[k];
            const int rmax = std::min(k + 2, hi);
            for (int i = l; i <= rmax; ++i) {
                const cd x = h(i, k), y = h(i, k + 1);
                h(i, k) = x * c + y * s;
                h(i, k + 1) = -x * std::conj(s) + y * std::conj(c);
            }
        }
        for (int k = l; k <= hi; ++k) h(k, k) += mu;
    }
    return (int)out.size() == n;
}

// LU with partial pivoting of an n x n matrix (row-major, in place); a zero
// pivot is replaced by `tiny` (inverse iteration at an exact eigenvalue).
template <typename T>
void lu(std::vector<T>& A, std::vector<int>& piv, int n, double tiny) {
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A[(size_t)i * n + k]) > best) {
                best = std::abs(A[(size_t)i * n + k]);
                p = i;
            }
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
        if (std::abs(A[(size_t)k * n + k]) == 0.0) A[(size_t)k * n + k] = T(tiny);
        const T inv = T(1.0) / A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const T f = A[(size_t)i * n + k] * inv;
            A[(size_t)i * n + k] = f;
            if (f != T(0.0))
                for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
        }
    }
}

template <typename T>
void lu_solve(const std::vector<T>& LU, const std::vector<int>& piv, int n, std::vector<T>& x) {
    for (int k = 0; k < n; ++k) std::swap(x[k], x[piv[k]]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) x[i] -= LU[(size_t)i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) x[i] -= LU[(size_t)i * n + j] * x[j];
        x[i] /= LU[(size_t)i * n + i];
    }
}

// conjugate that keeps real vectors real
inline double conjv(double v) { return v; }
inline cd conjv(cd v) { return std::conj(v); }

template <typename T>
double vnorm(const std::vector<T>& x) {
    double s = 0.0;
    for (const T& v : x) s += std::norm(cd(v));
    return std::sqrt(s);
}

// Inverse iteration for the eigenvector of Q (n x n) at shift sigma;
// `against` holds earlier vectors of the same cluster (orthogonalised away).
template <typename T>
std::vector<T> inverse_iteration(const std::vector<double>& Q, int n, T sigma, double scale, int seed,
                                 const std::vector<std::vector<T>>& against) {
    std::vector<T> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = T(Q[(size_t)i * n + j]) - (i == j ? sigma : T(0.0));
    std::vector<int> piv;
    lu(A, piv, n, 1e-14 * scale);
    std::vector<T> x(n);
    for (int i = 0; i < n; ++i) x[i] = T(1.0 + 0.37 * std::sin(1.3 * i + 0.7 * seed + 0.1));
    for (int it = 0; it < 4; ++it) {
        for (const auto& w : against) {
            T d = T(0.0);
            for (int i = 0; i < n; ++i) d += conjv(w[i]) * x[i];
            for (int i = 0; i < n; ++i) x[i] -= d * w[i];
        }
        lu_solve(A, piv, n, x);
        const double nx = vnorm(x);
        if (!(nx > 0.0) || !std::isfinite(nx)) return {};
        for (auto& v : x) v /= nx;
    }
    for (const auto& w : against) {
        T d = T(0.0);
        for (int i = 0; i < n; ++i) d += conjv(w[i]) * x[i];
        for (int i = 0; i < n; ++i) x[i] -= d * w[i];
    }
    const double nx = vnorm(x);
    if (!(nx > 0.0)) return {};
    for (auto& v : x) v /= nx;
    return x;
}

}  // namespace

bool eigen_decompose(int m, const double* Qin, EigenSystem& es) {
    const int n = m;
    es = EigenSystem{};
    es.m = m;
    std::vector<double> Q(Qin, Qin + (size_t)n * n);
    double scale = norm_inf(Q, n);
    if (scale == 0.0) scale = 1.0;
    std::vector<double> H = Q;
    hessenberg(H, n);
    std::vector<cd> lam;
    if (!hessenberg_eigenvalues(H, n, lam)) return false;

    // real eigenvalues and conjugate pairs
    const double im_tol = 1e-9 * scale;
    std::vector<double> reals;
    std::vector<cd> pos, neg;
    for (const cd& z : lam) {
        if (std::fabs(z.imag()) <= im_tol) reals.push_back(z.real());
        else if (z.imag() > 0) pos.push_back(z);
        else neg.push_back(z);
    }
    if (pos.size() != neg.size()) return false;
    std::vector<cd> pairs;
    std::vector<bool> used(neg.size(), false);
    for (const cd& z : pos) {
        int best = -1;
        double bd = 0.0;
        for (size_t k = 0; k < neg.size(); ++k)
            if (!used[k]) {
                const double d = std::abs(z - std::conj(neg[k]));
                if (best < 0 || d < bd) {
                    best = (int)k;
                    bd = d;
                }
            }
        if (best < 0 || bd > 1e-6 * scale) return false;
        used[best] = true;
        pairs.push_back(0.5 * (z + std::conj(neg[best])));
    }
    std::sort(reals.begin(), reals.end());
    std::sort(pairs.begin(), pairs.end(), [](const cd& a, const cd& b) {
        return a.real() != b.real() ? a.real() < b.real() : a.imag() < b.imag();
    });

    es.V.assign((size_t)n * n, 0.0);
    es.re.assign(n, 0.0);
    es.im.assign(n, 0.0);
    es.kind.assign(n, 0);
    int col = 0;
    const double clus = 1e-7 * scale;
    {
        std::vector<std::vector<double>> cluster;
        double last = 0.0;
        for (size_t r = 0; r < reals.size(); ++r) {
            const double z = reals[r];
            if (r == 0 || std::fabs(z - last) > clus) cluster.clear();
            last = z;
            const double sigma = z + 1e-10 * scale;
            std::vector<double> x = inverse_iteration<double>(Q, n, sigma, scale, (int)r, cluster);
            if (x.empty()) return false;
            cluster.push_back(x);
            for (int i = 0; i < n; ++i) es.V[(size_t)i * n + col] = x[i];
            es.re[col] = z;
            es.kind[col] = 0;
            ++col;
        }
    }
    {
        std::vector<std::vector<cd>> cluster;
        cd last = 0.0;
        for (size_t r = 0; r < pairs.size(); ++r) {
            const cd z = pairs[r];
            if (r == 0 || std::abs(z - last) > clus) cluster.clear();
            last = z;
            const cd sigma = z + cd(1e-10 * scale, 0.0);
            std::vector<cd> x = inverse_iteration<cd>(Q, n, sigma, scale, (int)r + 101, cluster);
            if (x.empty()) return false;
            cluster.push_back(x);
            // phase that makes the real and imaginary parts orthogonal
            cd s2 = 0.0;
            for (const cd& v : x) s2 += v * v;
            const cd rot = std::polar(1.0, -0.5 * std::arg(s2));
            for (int i = 0; i < n; ++i) {
                const cd v = x[i] * rot;
                es.V[(size_t)i * n + col] = v.real();
                es.V[(size_t)i * n + col + 1] = v.imag();
            }
            es.re[col] = es.re[col + 1] = z.real();
            es.im[col] = es.im[col + 1] = z.imag();
            es.kind[col] = 1;
            es.kind[col + 1] = 2;
            col += 2;
        }
    }
    if (col != n) return false;

    // V^-1
    std::vector<double> LU = es.V;
    std::vector<int> piv;
    lu(LU, piv, n, 0.0);
    for (int k = 0; k < n; ++k)
        if (LU[(size_t)k * n + k] == 0.0 || !std::isfinite(LU[(size_t)k * n + k])) return false;
    es.Vinv.assign((size_t)n * n, 0.0);
    std::vector<double> e(n);
    for (int j = 0; j < n; ++j) {
        std::fill(e.begin(), e.end(), 0.0);
        e[j] = 1.0;
        lu_solve(LU, piv, n, e);
        for (int i = 0; i < n; ++i) es.Vinv[(size_t)i * n + j] = e[i];
    }
    auto norm1 = [&](const std::vector<double>& A) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += std::fabs(A[(size_t)i * n + j]);
            r = std::max(r, s);
        }
        return r;
    };
    es.cond = norm1(es.V) * norm1(es.Vinv);

    // reconstruction V B V^-1 against Q
    std::vector<double> VB((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v;
            if (es.kind[j] == 0) v = es.V[(size_t)i * n + j] * es.re[j];
            else if (es.kind[j] == 1)  // column j: a v_r - b v_i
                v = es.re[j] * es.V[(size_t)i * n + j] - es.im[j] * es.V[(size_t)i * n + j + 1];
            else  // column j (second of the pair): b v_r + a v_i
                v = es.im[j] * es.V[(size_t)i * n + j - 1] + es.re[j] * es.V[(size_t)i * n + j];
            VB[(size_t)i * n + j] = v;
        }
    double qmax = 0.0, err = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += VB[(size_t)i * n + k] * es.Vinv[(size_t)k * n + j];
            err = std::max(err, std::fabs(acc - Q[(size_t)i * n + j]));
            qmax = std::max(qmax, std::fabs(Q[(size_t)i * n + j]));
        }
    es.resid = err / (qmax > 0.0 ? qmax : 1.0);
    return std::isfinite(es.cond) && std::isfinite(es.resid);
}

}  // namespace pg
