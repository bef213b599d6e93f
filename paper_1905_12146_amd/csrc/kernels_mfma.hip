// Split-BF16 kernels for large state spaces (any m <= 64, padded to MP = 64;
// meant for 61-state codon models): every product of a transition matrix,
// or of Q, with a partial vector runs on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; partial vectors are
// FP32.  The passes compute the same quantities as the FP64 / FP32 kernels
// (Sections 2.3-2.6): post-order messages m_k = P_k p~_k, per-category root
// values and scale exponents, pre-order vectors q and the per-branch ratio
// (u^T Q m) / (u^T m) weighted by w_s rho_{s,l} gamma_l.
//
// Tile and register layout.  A wave owns one tile (16 consecutive patterns
// of one category) of one node at a time.  A vector of MP states x 16
// patterns is the 64 x 16 B operand / accumulator of the MFMA: lane
// L = 16 g + c holds pattern c and states 16 mt + 4 g + i (mt, i = 0..3),
// exactly its four f32x4 accumulators D[mt].  The contraction index (the
// state y of the vector) is ordered as
//   k slot (ks, g, j)  ->  state 16 (2 ks + j / 4) + 4 g + j % 4,
// so the B operand of k-step ks is the lane's own values of blocks 2 ks and
// 2 ks + 1: a product's output feeds the next product from registers, with
// no exchange between lanes.  A fragments are stored in the same order.
// In HBM one tile of a vector is the lanes' f32x4 in order,
// [node][tile][mt][lane], read and written as whole-wave 1 KB runs.
//
// Split products.  An FP32 operand x is carried as three BF16 parts,
// x = x_hi + x_mid + x_lo (x_hi = bf16(x), x_mid = bf16(x - x_hi), x_lo =
// bf16(x - x_hi - x_mid): the full 24-bit significand), and A x is the sum
// of the six part products of order >= 2^-16 relative (hi hi, hi mid,
// mid hi, hi lo, mid mid, lo hi), each on the matrix cores with FP32
// accumulation, smallest first.  Transition matrices enter as F = P - I:
// the accumulator starts at x (exact) and the MFMAs add F x, so rounding
// scales with |F|.  Q x (gradient numerator) cancels between the diagonal
// and the off-diagonal rates; Q is split the same way.  (With two parts per
// operand and three products the error is ~2^-16 |F| |x|, which on long
// branches, where the gradient is exponentially small, exceeds 1e-5 of it.)
//
// Transition matrices, per (branch, category), in FP64:
//   F = V (exp(B gamma_l t_b) - I) V^-1     eigen route, one product, or
//   F by scaling and squaring of the Taylor series (Q not usably
//   diagonalisable),
// then written as operands: for an internal branch the A fragments (hi, mid,
// lo) of F (post-order) and F^T (pre-order); for a tip branch the FP32 table of
// P's columns (row y = P[.][y]; row MP = P 1 for the fully ambiguous code).
#include "device_common.h"

namespace pg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MW = 8;                // waves per traversal workgroup
constexpr int MF_THREADS = MW * 64;
constexpr int MF_TAYLOR_DEG = 16;

struct V16 {
    f32x4 v[4];
};

__device__ inline size_t mvec_off(const EvalArgs& a, int node, int tile) {
    return ((size_t)(node - a.n_tips) * a.n_tiles + tile) * (size_t)(MP * TP);
}

__device__ inline const char* slot_of(const EvalArgs& a, int b, int l) {
    return static_cast<const char*>(a.P) + ((size_t)b * a.K + l) * MF_SLOT_BYTES;
}

// A fragments of F (which = 0) or F^T (which = 1) of branch b, category l:
// [mt][ks][part][lane], part 0 = hi, 1 = mid, 2 = lo.
constexpr int FRAGS = 8 * 3 * 64;  // bf16x8 per matrix
__device__ inline const bf16x8* frag_of(const EvalArgs& a, int b, int l, int which) {
    return reinterpret_cast<const bf16x8*>(slot_of(a, b, l)) + which * FRAGS;
}

__device__ inline void vload(const float* base, int lane, V16& r) {
    const f32x4* src = reinterpret_cast<const f32x4*>(base);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) r.v[mt] = src[mt * 64 + lane];
}

__device__ inline void vstore(float* base, int lane, const V16& r) {
    f32x4* dst = reinterpret_cast<f32x4*>(base);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) dst[mt * 64 + lane] = r.v[mt];
}

// reductions over the four lane groups g holding the same pattern; every
// lane gets the same bits ((g0 + g1) + (g2 + g3) in either operand order)
__device__ inline float xmax4(float v) {
    v = fmaxf(v, __shfl_xor(v, 16));
    return fmaxf(v, __shfl_xor(v, 32));
}
__device__ inline float xsum4(float v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
}
__device__ inline double xsum4(double v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// B operands of x in three BF16 parts.
__device__ inline void split3(const V16& x, bf16x8 hi[2], bf16x8 mid[2], bf16x8 lo[2]) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float v = x.v[2 * ks + j / 4][j % 4];
            const __bf16 h = (__bf16)v;
            const float r1 = v - (float)h;
            const __bf16 m = (__bf16)r1;
            hi[ks][j] = h;
            mid[ks][j] = m;
            lo[ks][j] = (__bf16)(r1 - (float)m);
        }
}

// acc += A x, A given by its (hi, mid, lo) fragments [mt][ks][part][lane]
// (F or F^T in global memory, Q in LDS).  The four row blocks interleave so
// consecutive MFMAs are independent.
__device__ inline void apply3(const bf16x8* __restrict__ A, int lane, const V16& x, V16& acc) {
    bf16x8 xh[2], xm[2], xl[2];
    split3(x, xh, xm, xl);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x8 ah[4], am[4], al[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            ah[mt] = A[((mt * 2 + ks) * 3 + 0) * 64 + lane];
            am[mt] = A[((mt * 2 + ks) * 3 + 1) * 64 + lane];
            al[mt] = A[((mt * 2 + ks) * 3 + 2) * 64 + lane];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(al[mt], xh[ks], acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(am[mt], xm[ks], acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ah[mt], xl[ks], acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(am[mt], xh[ks], acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ah[mt], xm[ks], acc.v[mt]);
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x8 ah[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ah[mt] = A[((mt * 2 + ks) * 3 + 0) * 64 + lane];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ah[mt], xh[ks], acc.v[mt]);
    }
}

// Outgoing message of child c (Section 2.1): the stored m_c of an internal
// child; for a tip, P_c times the tip indicator: one row of the tip table
// (observed state, or the all-ones row), or the sum of the allowed rows.
__device__ inline void child_vec(const EvalArgs& a, int c, int l, int tile, int s, int lane, V16& out) {
    if (c >= a.n_tips) {
        vload(static_cast<const float*>(a.msg) + mvec_off(a, c, tile), lane, out);
        return;
    }
    const int g = lane >> 4;
    const unsigned code = a.codes[(size_t)c * a.S_pad + s];
    const float* T = reinterpret_cast<const float*>(slot_of(a, c, l)) + 4 * g;
    const int row = code < (unsigned)a.M ? (int)code : (code == 255u ? MP : -1);
    if (row >= 0) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) out.v[mt] = *reinterpret_cast<const f32x4*>(T + row * MP + 16 * mt);
    } else {
        const unsigned long long mask = a.masks[code];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) out.v[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int y = 0; y < a.M; ++y)
            if ((mask >> y) & 1ull) {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) out.v[mt] += *reinterpret_cast<const f32x4*>(T + y * MP + 16 * mt);
            }
    }
}

// Scale v by 2^-e, e the exponent of its largest entry over the pattern's
// states; returns e (0 for an all-zero vector).
__device__ inline int rescale(V16& v) {
    float mx = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) mx = fmaxf(mx, v.v[mt][i]);
    mx = xmax4(mx);
    if (!(mx > 0.f)) return 0;
    const int e = exp_of(mx);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) v.v[mt][i] = ldexpf(v.v[mt][i], -e);
    return e;
}

// ---------------------------------------------------------------- transition matrices

__device__ inline bool mf_bad_length(double t) { return !(t >= 0.0) || isinf(t); }

// 4 x 4 block of C = A B with A and B in LDS (row-major, padded rows).
__device__ inline void block_product(const double (*A)[MP + 1], const double (*B)[MP + 1], int x0, int y0,
                                     double acc[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < MP; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = A[x0 + i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = B[k][y0 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
}

__device__ inline void mfma_pmat_body(const EvalArgs& a, int block) {
    __shared__ double Fs[MP][MP + 1];
    __shared__ double Ws[MP][MP + 1];
    const int b = block / a.K, l = block % a.K;
    const int tid = threadIdx.x;
    const int x0 = 4 * (tid / 16), y0 = 4 * (tid % 16);
    const int M = a.M;
    const double tb = a.t[b];
    const bool bad = mf_bad_length(tb);
    double acc[4][4];
    if (!bad && !a.expm_taylor) {
        // Fs = V (exp(B tau) - I), Ws = V^-1, F = Fs Ws
        const double tau = a.rates[l] * tb;
        for (int e = tid; e < MP * MP; e += blockDim.x) {
            const int x = e / MP, j = e % MP;
            const int kind = a.eKind[j];
            double v;
            if (kind == 0) {
                v = a.eV[e] * expm1(a.eRe[j] * tau);
            } else {
                const double ar = a.eRe[j] * tau, bi = a.eIm[j] * tau;
                const double sh = sin(0.5 * bi);
                const double C = expm1(ar) * cos(bi) - 2.0 * sh * sh;  // e^ar cos(bi) - 1
                const double S = exp(ar) * sin(bi);
                v = (kind == 1) ? a.eV[e] * C - a.eV[e + 1] * S : a.eV[e - 1] * S + a.eV[e] * C;
            }
            Fs[x][j] = v;
            Ws[x][j] = a.eVinv[e];
        }
        __syncthreads();
        block_product(Fs, Ws, x0, y0, acc);
    } else if (!bad) {
        // F = exp(A) - I, A = Q rate t 2^-s with ||A||_inf <= 1/2:
        //   G = I + A/2 (I + A/3 (... (I + A/DEG))), F = A G, then s times
        //   F <- 2F + F F.  A is read from Q in global memory; G (then F)
        //   lives in Fs.
        const double h = a.rates[l] * tb;
        double nrm = a.qnorm * h;
        int sq = 0;
        while (nrm > 0.5 && sq < 1100) {
            nrm *= 0.5;
            ++sq;
        }
        const double hs = ldexp(h, -sq);
        auto a_entry = [&](int x, int y) { return (x < M && y < M) ? a.Q64[x * M + y] * hs : 0.0; };
        for (int e = tid; e < MP * MP; e += blockDim.x) Fs[e / MP][e % MP] = (e / MP == e % MP) ? 1.0 : 0.0;
        __syncthreads();
        auto times_a = [&](double out[4][4]) {  // out = A Fs (own block)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) out[i][j] = 0.0;
            for (int k = 0; k < MP; ++k) {
                double av[4], bv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) av[i] = a_entry(x0 + i, k);
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = Fs[k][y0 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) out[i][j] = fma(av[i], bv[j], out[i][j]);
            }
        };
        for (int k = MF_TAYLOR_DEG; k >= 2; --k) {
            times_a(acc);
            __syncthreads();
            const double inv = 1.0 / k;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) Fs[x0 + i][y0 + j] = ((x0 + i == y0 + j) ? 1.0 : 0.0) + acc[i][j] * inv;
            __syncthreads();
        }
        times_a(acc);  // F
        for (int r = 0; r < sq; ++r) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) Fs[x0 + i][y0 + j] = acc[i][j];
            __syncthreads();
            double f2[4][4];
            block_product(Fs, Fs, x0, y0, f2);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = 2.0 * acc[i][j] + f2[i][j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) Fs[x0 + i][y0 + j] = bad ? (double)NAN : acc[i][j];
    __syncthreads();

    char* slot = static_cast<char*>(a.P) + ((size_t)b * a.K + l) * MF_SLOT_BYTES;
    if (b >= a.n_tips) {
        // A fragments [which][mt][ks][part][lane] of F (which 0) and F^T (1)
        bf16x8* out = reinterpret_cast<bf16x8*>(slot);
        for (int c = tid; c < 2 * FRAGS; c += blockDim.x) {
            const int L = c % 64, part = (c / 64) % 3, ks = (c / 192) % 2, mt = (c / 384) % 4, which = c / FRAGS;
            const int r = 16 * mt + L % 16, g = L / 16;
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int y = 16 * (2 * ks + j / 4) + 4 * g + j % 4;
                const double f = which == 0 ? Fs[r][y] : Fs[y][r];
                const __bf16 hi = (__bf16)(float)f;
                const double r1 = f - (double)(float)hi;
                const __bf16 mid = (__bf16)(float)r1;
                v[j] = part == 0 ? hi : part == 1 ? mid : (__bf16)(float)(r1 - (double)(float)mid);
            }
            out[c] = v;
        }
    } else {
        // tip table: row y < MP = column y of P, row MP = P 1
        float* T = reinterpret_cast<float*>(slot);
        for (int e = tid; e < (MP + 1) * MP; e += blockDim.x) {
            const int y = e / MP, x = e % MP;
            float v = 0.f;
            if (x < M) {
                if (y < M) {
                    v = (float)(((x == y) ? 1.0 : 0.0) + Fs[x][y]);
                } else if (y == MP) {
                    double sum = 0.0;
                    for (int z = 0; z < M; ++z) sum += Fs[x][z];
                    v = (float)(1.0 + sum);
                }
            }
            T[e] = v;
        }
    }
}

// ---------------------------------------------------------------- post-order pass

__device__ inline void mfma_post_body(const EvalArgs& a, int tile, int4* lds_sched) {
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ps = lane & 15, g = lane >> 4;
    const int s = pb * TP + ps;
    stage_schedule(a, lds_sched);
    int esum = 0;
    for (int h = 0; h < a.n_levels; ++h) {
        const int end = a.level_off[h + 1];
        for (int idx = a.level_off[h] + wv; idx < end; idx += MW) {
            const int4 nd = sched_at(a, lds_sched, idx);
            V16 mi, mj, p;
            child_vec(a, nd.y, l, tile, s, lane, mi);
            child_vec(a, nd.z, l, tile, s, lane, mj);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) p.v[mt] = mi.v[mt] * mj.v[mt];
            esum += rescale(p);
            if (nd.x != a.root) {
                V16 acc = p;
                apply3(frag_of(a, nd.x, l, 0), lane, p, acc);
                vstore(static_cast<float*>(a.msg) + mvec_off(a, nd.x, tile), lane, acc);
            } else {
                double Lt = 0.0;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int x = 16 * mt + 4 * g + i;
                        if (x < a.M) Lt = fma(a.pi64[x], (double)p.v[mt][i], Lt);
                    }
                Lt = xsum4(Lt);
                if (g == 0) a.rootL[(size_t)l * a.S_pad + s] = Lt;
            }
        }
        __syncthreads();
    }
    __shared__ int red[MW][TP];
    if (g == 0) red[wv][ps] = esum;
    __syncthreads();
    if (wv == 0 && g == 0) {
        int tot = 0;
        for (int i = 0; i < MW; ++i) tot += red[i][ps];
        a.rootE[(size_t)l * a.S_pad + s] = tot;
    }
}

// ---------------------------------------------------------------- pre-order pass + gradient

// Child c with sibling message msib under a node with pre-order vector q:
//   u = q o msib, ratio = (u^T Q m_c) / (u^T m_c), tile sum of g * ratio,
//   and for an internal c: q_c = P_c^T u = u + F_c^T u, rescaled, stored.
__device__ inline void mfma_pre_child(const EvalArgs& a, int c, int l, int tile, int lane, const Coef& cf,
                                      const V16& q, const V16& msib, const V16& mown, const bf16x8* qop) {
    V16 u;
    float den = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        u.v[mt] = q.v[mt] * msib.v[mt];
#pragma unroll
        for (int i = 0; i < 4; ++i) den = fmaf(u.v[mt][i], mown.v[mt][i], den);
    }
    V16 qm;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) qm.v[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    apply3(qop, lane, mown, qm);
    float num = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) num = fmaf(u.v[mt][i], qm.v[mt][i], num);
    den = xsum4(den);
    num = xsum4(num);
    const double ratio = (den > 0.f) ? (double)num / (double)den : 0.0;
    double term = (cf.g > 0.0) ? cf.g * ratio : 0.0;
    term = sum16(term);  // every row holds the same 16 patterns
    if (lane == 0) a.partial[(size_t)tile * a.n_branches + c] = term;
    if (c >= a.n_tips) {
        V16 acc = u;
        apply3(frag_of(a, c, l, 1), lane, u, acc);
        (void)rescale(acc);
        vstore(static_cast<float*>(a.qv) + mvec_off(a, c, tile), lane, acc);
    }
}

__device__ inline void mfma_pre_body(const EvalArgs& a, int tile, int4* lds_sched) {
    __shared__ bf16x8 qop[3 * 8 * 64];
    const int l = tile / a.n_pb, pb = tile % a.n_pb;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ps = lane & 15, g = lane >> 4;
    const int s = pb * TP + ps;
    Coef cf;
    {
        const SiteLik r = site_likelihood(a, s);
        cf = coef_of(a, l, s, r);
        // the category-0 tile of each pattern block also forms its logL part
        if (l == 0 && wv == 0 && g == 0) logl_block_part(a, pb, ps, r);
    }
    const bf16x8* qsrc = static_cast<const bf16x8*>(a.Qop);
    for (int i = threadIdx.x; i < 3 * 8 * 64; i += blockDim.x) qop[i] = qsrc[i];
    stage_schedule(a, lds_sched);
    __syncthreads();
    V16 piv;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = 16 * mt + 4 * g + i;
            piv.v[mt][i] = x < a.M ? (float)a.pi64[x] : 0.f;
        }
    for (int h = a.n_levels - 1; h >= 0; --h) {
        const int end = a.level_off[h + 1];
        for (int idx = a.level_off[h] + wv; idx < end; idx += MW) {
            const int4 nd = sched_at(a, lds_sched, idx);
            V16 q, mi, mj;
            if (nd.x == a.root) q = piv;
            else vload(static_cast<const float*>(a.qv) + mvec_off(a, nd.x, tile), lane, q);
            child_vec(a, nd.y, l, tile, s, lane, mi);
            child_vec(a, nd.z, l, tile, s, lane, mj);
            mfma_pre_child(a, nd.y, l, tile, lane, cf, q, mj, mi, qop);
            mfma_pre_child(a, nd.z, l, tile, lane, cf, q, mi, mj, qop);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- entry points

__global__ void __launch_bounds__(256) mfma_pmat_kernel(EvalArgs a) { mfma_pmat_body(a, blockIdx.x); }

__global__ void __launch_bounds__(MF_THREADS) mfma_post_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    mfma_post_body(a, blockIdx.x, lds_dyn);
}

__global__ void __launch_bounds__(MF_THREADS) mfma_pre_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    mfma_pre_body(a, blockIdx.x, lds_dyn);
}

size_t mfma_post_lds_bytes(const EvalArgs& a) { return sched_lds_bytes(a); }
size_t mfma_pre_lds_bytes(const EvalArgs& a) { return sched_lds_bytes(a); }

hipError_t launch_mfma_pmat(const EvalArgs& a, hipStream_t st) {
    mfma_pmat_kernel<<<a.n_branches * a.K, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mfma_post(const EvalArgs& a, hipStream_t st) {
    mfma_post_kernel<<<a.n_tiles, MF_THREADS, mfma_post_lds_bytes(a), st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mfma_pre(const EvalArgs& a, hipStream_t st) {
    mfma_pre_kernel<<<a.n_tiles, MF_THREADS, mfma_pre_lds_bytes(a), st>>>(a);
    return hipGetLastError();
}

}  // namespace pg
