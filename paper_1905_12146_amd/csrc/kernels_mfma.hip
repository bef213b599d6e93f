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

// acc += A x, A given by its (hi, mid, lo) fragments [mt][ks][part][lane]
// (F or F^T in global memory, Q in LDS).  Per k-step the parts are loaded
// one at a time (lo, mid, hi) so only 16 registers of A are live; the four
// row blocks interleave so consecutive MFMAs are independent.  Order per
// k-step: lo*hi, mid*mid, mid*hi, hi*lo, hi*mid, hi*hi (smallest first).
// FENCE (A in global memory): keep each part's loads next to its MFMAs
// (hoisted ahead, the loads of all parts would hold 96 registers).
template <bool FENCE = false>
__device__ inline void apply3(const bf16x8* __restrict__ A, int lane, const V16& x, V16& acc) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x8 xh, xm, xl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float v = x.v[2 * ks + j / 4][j % 4];
            const __bf16 h = (__bf16)v;
            const float r1 = v - (float)h;  // exact in FP32
            const __bf16 m = (__bf16)r1;
            xh[j] = h;
            xm[j] = m;
            xl[j] = (__bf16)(r1 - (float)m);
        }
        bf16x8 ap[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ap[mt] = A[((mt * 2 + ks) * 3 + 2) * 64 + lane];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xh, acc.v[mt]);
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ap[mt] = A[((mt * 2 + ks) * 3 + 1) * 64 + lane];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xm, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xh, acc.v[mt]);
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ap[mt] = A[((mt * 2 + ks) * 3 + 0) * 64 + lane];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xl, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xm, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(ap[mt], xh, acc.v[mt]);
    }
}

// The 24 A fragments of one 64 x 64 matrix in registers ([ks][part][mt]),
// issued together so a product waits for one memory round trip.
struct Frags {
    bf16x8 f[2][3][4];
};

__device__ inline void frags_issue(const bf16x8* __restrict__ A, int lane, Frags& F) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int part = 0; part < 3; ++part)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) F.f[ks][part][mt] = A[((mt * 2 + ks) * 3 + part) * 64 + lane];
}

// acc += A x with A's fragments in registers; same products and order as
// apply3.
__device__ inline void apply3f(const Frags& F, const V16& x, V16& acc) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        bf16x8 xh, xm, xl;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float v = x.v[2 * ks + j / 4][j % 4];
            const __bf16 h = (__bf16)v;
            const float r1 = v - (float)h;
            const __bf16 m = (__bf16)r1;
            xh[j] = h;
            xm[j] = m;
            xl[j] = (__bf16)(r1 - (float)m);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][2][mt], xh, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][1][mt], xm, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][1][mt], xh, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][0][mt], xl, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][0][mt], xm, acc.v[mt]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc.v[mt] = mfma(F.f[ks][0][mt], xh, acc.v[mt]);
    }
}

// Outgoing message of child c (Section 2.1): the stored m_c of an internal
// child; for a tip, P_c times the tip indicator: one row of the tip table
// (observed state, or the all-ones row), or the sum of the allowed rows.
// Split in two so a node's loads can be issued one node ahead:
// child_issue loads the message (internal) or the tip code, child_finish
// reads the tip table.
struct ChildLd {
    V16 v;
    unsigned code;
};

__device__ inline void child_issue(const EvalArgs& a, int c, int tile, int s, int lane, ChildLd& r) {
    if (c >= a.n_tips) vload(static_cast<const float*>(a.msg) + mvec_off(a, c, tile), lane, r.v);
    else r.code = a.codes[(size_t)c * a.S_pad + s];
}

__device__ inline void child_finish(const EvalArgs& a, int c, int l, int lane, const ChildLd& r, V16& out) {
    if (c >= a.n_tips) {
        out = r.v;
        return;
    }
    const int g = lane >> 4;
    const unsigned code = r.code;
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

typedef double d4 __attribute__((ext_vector_type(4)));

// C = A B for 64 x 64 FP64 matrices in LDS (row-major, padded rows) on the
// matrix cores (v_mfma_f64_16x16x4f64), by a workgroup of 4 waves: wave w
// forms rows 16w..16w+15 (four 16 x 16 tiles), k in steps of 4 (operand
// lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k).  After a
// barrier each lane writes out[x][y] = epi(x, y, C[x][y]) for its own
// elements (item r of tile t at lane j + 16g is row g + 4r, column j), so
// out may be A or B; ends with a barrier.
template <typename Epi>
__device__ inline void lds_product(const double (*A)[MP + 1], const double (*B)[MP + 1], double (*out)[MP + 1],
                                   Epi epi) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, kk = lane >> 4;
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = 0; k0 < MP; k0 += 4) {
        const double av = A[16 * w + i][k0 + kk];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, B[k0 + kk][16 * t + i], acc[t], 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = 16 * w + kk + 4 * r, y = 16 * t + i;
            out[x][y] = epi(x, y, acc[t][r]);
        }
    __syncthreads();
}

__device__ inline void mfma_pmat_body(const EvalArgs& a, int block) {
    __shared__ double Fs[MP][MP + 1];
    __shared__ double Ws[MP][MP + 1];
    __shared__ double fc[MP], fsn[MP];
    const int b = a.blist ? a.blist[block / a.K] : block / a.K, l = block % a.K;
    const int tid = threadIdx.x;
    const int M = a.M;
    const double tb = a.t[b];
    const bool bad = mf_bad_length(tb);
    auto keep = [](int, int, double c) { return c; };
    if (!bad && !a.expm_taylor && a.n_models == 0) {
        // F = V X with X = (exp(B tau) - I) V^-1: row j of X is
        //   C_j r_j                      (real eigenvalue, C = expm1(re tau))
        //   C r_j + S r_{j+1}, -S r_j + C r_{j+1}   (pair j, j+1; C = e^{a} cos b
        //                                 - 1, S = e^{a} sin b with a, b = re, im x tau)
        // where r_j is row j of V^-1.
        const double tau = a.rates[l] * tb;
        if (tid < MP) {
            const int kind = a.eKind[tid];
            const double ar = a.eRe[tid] * tau;
            double C, S = 0.0;
            if (kind == 0) {
                C = expm1(ar);
            } else {
                const double bi = a.eIm[tid] * tau;
                const double sh = sin(0.5 * bi);
                C = expm1(ar) * cos(bi) - 2.0 * sh * sh;
                S = exp(ar) * sin(bi);
            }
            fc[tid] = C;
            fsn[tid] = kind == 1 ? S : kind == 2 ? -S : 0.0;  // coefficient of the partner row
        }
        double vv[16], wv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            vv[i] = a.eV[tid + 256 * i];
            wv[i] = a.eVinv[tid + 256 * i];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            Fs[e / MP][e % MP] = vv[i];
            Ws[e / MP][e % MP] = wv[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i, j = e / MP, y = e % MP;
            const int kind = a.eKind[j];
            const int partner = kind == 1 ? j + 1 : kind == 2 ? j - 1 : j;
            wv[i] = fc[j] * Ws[j][y] + fsn[j] * Ws[partner][y];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            Ws[e / MP][e % MP] = wv[i];
        }
        __syncthreads();
        lds_product(Fs, Ws, Fs, keep);  // F = V X
    } else if (!bad) {
        // F = exp(A) - I, A = Q rate t 2^-s with ||A||_inf <= 1/2:
        //   G = I + A/2 (I + A/3 (... (I + A/DEG))), F = A G, then s times
        //   F <- 2F + F F.  A is staged in Ws, G (then F) lives in Fs.
        const double h = a.rates[l] * tb;
        // the model's rate matrix, or branch b's own (non-homogeneous model)
        const double* Qb = a.n_models ? a.Qm + (size_t)a.branch_model[b] * M * M : a.Q64;
        double nrm = (a.n_models ? a.qnorm_m[a.branch_model[b]] : a.qnorm) * h;
        int sq = 0;
        while (nrm > 0.5 && sq < 1100) {
            nrm *= 0.5;
            ++sq;
        }
        const double hs = ldexp(h, -sq);
        for (int e = tid; e < MP * MP; e += blockDim.x) {
            const int x = e / MP, y = e % MP;
            Ws[x][y] = (x < M && y < M) ? Qb[x * M + y] * hs : 0.0;
            Fs[x][y] = (x == y) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int k = MF_TAYLOR_DEG; k >= 2; --k) {
            const double inv = 1.0 / k;
            lds_product(Ws, Fs, Fs, [inv](int x, int y, double c) { return ((x == y) ? 1.0 : 0.0) + c * inv; });
        }
        lds_product(Ws, Fs, Fs, keep);  // F
        for (int r = 0; r < sq; ++r)
            lds_product(Fs, Fs, Fs, [&](int x, int y, double c) { return 2.0 * Fs[x][y] + c; });
    }
    if (bad) {
        for (int e = tid; e < MP * MP; e += blockDim.x) Fs[e / MP][e % MP] = (double)NAN;
        __syncthreads();
    }

    char* slot = static_cast<char*>(a.P) + ((size_t)b * a.K + l) * MF_SLOT_BYTES;
    if (b >= a.n_tips) {
        // A fragments [which][mt][ks][part][lane] of F (which 0) and F^T (1);
        // each thread splits 8 entries once and writes their three parts
        bf16x8* out = reinterpret_cast<bf16x8*>(slot);
        for (int c = tid; c < 2 * 8 * 64; c += blockDim.x) {
            const int L = c % 64, ks = (c / 64) % 2, mt = (c / 128) % 4, which = c / 512;
            const int r = 16 * mt + L % 16, g = L / 16;
            bf16x8 vh, vm, vl;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int y = 16 * (2 * ks + j / 4) + 4 * g + j % 4;
                const double f = which == 0 ? Fs[r][y] : Fs[y][r];
                const __bf16 hi = (__bf16)(float)f;
                const double r1 = f - (double)(float)hi;
                const __bf16 mid = (__bf16)(float)r1;
                vh[j] = hi;
                vm[j] = mid;
                vl[j] = (__bf16)(float)(r1 - (double)(float)mid);
            }
            bf16x8* dst = out + which * FRAGS + (mt * 2 + ks) * 3 * 64 + L;
            dst[0] = vh;
            dst[64] = vm;
            dst[128] = vl;
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

// One internal node k of the post-order pass for this wave's tile:
//   p_k = m_i o m_j, rescaled; m_k = p_k + F_k p_k stored (k not the root)
//   or the root value pi^T p~ (Eq. rootInnerProduct).
__device__ inline void mfma_post_node(const EvalArgs& a, int4 nd, int l, int tile, int s, int lane,
                                      const ChildLd& ci, const ChildLd& cj, int& esum) {
    const int g = lane >> 4;
    const bool has_msg = nd.x != a.root;
    Frags F;
    if (has_msg) frags_issue(frag_of(a, nd.x, l, 0), lane, F);  // with the tip-table loads
    V16 mi, mj, p;
    child_finish(a, nd.y, l, lane, ci, mi);
    child_finish(a, nd.z, l, lane, cj, mj);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) p.v[mt] = mi.v[mt] * mj.v[mt];
    const int e = rescale(p);
    if (a.expo) {
        // per-node exponents for partial re-evaluation (lane group 0 owns
        // them): a pass over some nodes adds the change of each visited
        // node's exponent
        if (g == 0) {
            int16_t* ex = a.expo + ((size_t)(nd.x - a.n_tips) * a.n_tiles + tile) * TP + (lane & 15);
            esum += a.expo_delta ? e - (int)*ex : e;
            *ex = (int16_t)e;
        }
    } else {
        esum += e;
    }
    if (has_msg) {
        V16 acc = p;
        apply3f(F, p, acc);
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

__device__ inline void mfma_post_body(const EvalArgs& a, int tile, int4* lds_sched) {
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
            ChildLd ci, cj;
            child_issue(a, nd.y, tile, s, lane, ci);
            child_issue(a, nd.z, tile, s, lane, cj);
            while (true) {
                const int nidx = idx + MW;
                const bool more = nidx < end;
                int4 nn = nd;
                ChildLd ni, nj;
                if (more) {
                    nn = sched_at(a, lds_sched, nidx);
                    child_issue(a, nn.y, tile, s, lane, ni);
                    child_issue(a, nn.z, tile, s, lane, nj);
                }
                mfma_post_node(a, nd, l, tile, s, lane, ci, cj, esum);
                if (!more) break;
                nd = nn;
                ci = ni;
                cj = nj;
                idx = nidx;
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
        if (a.expo_delta) a.rootE[(size_t)l * a.S_pad + s] += tot;
        else a.rootE[(size_t)l * a.S_pad + s] = tot;
    }
}

// ---------------------------------------------------------------- pre-order pass + gradient

// Child c under a node, with its top-of-branch vector u = q o m_sibling:
//   ratio = (u^T Q m_c) / (u^T m_c), tile sum of g * ratio,
//   and for an internal c: q_c = P_c^T u = u + F_c^T u, rescaled, stored
// (F holds F_c^T's fragments, issued by the caller).  HESS adds, for
// Section 2.7, the tile sum of h * (u^T Q^2 m_c) / (u^T m_c) and the
// per-pattern rho gamma ratio (reduced by hsum_kernel); Q^2's fragments
// are staged in LDS like Q's.
template <bool HESS, bool NH = false>
__device__ inline void mfma_pre_child(const EvalArgs& a, int c, int l, int tile, int s, int lane, const Coef& cf,
                                      const V16& u, const V16& mown, const bf16x8* qop, const bf16x8* q2op,
                                      Frags& F) {
    float den = 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) den = fmaf(u.v[mt][i], mown.v[mt][i], den);
    V16 qm;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) qm.v[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    apply3<NH>(qop, lane, mown, qm);
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
    if constexpr (HESS) {
        V16 q2m;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) q2m.v[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        apply3<NH>(q2op, lane, mown, q2m);
        float num2 = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) num2 = fmaf(u.v[mt][i], q2m.v[mt][i], num2);
        num2 = xsum4(num2);
        const double ratio2 = (den > 0.f) ? (double)num2 / (double)den : 0.0;
        double term2 = (cf.h > 0.0) ? cf.h * ratio2 : 0.0;
        term2 = sum16(term2);
        if (lane == 0) a.partial2[(size_t)tile * a.n_branches + c] = term2;
        if ((lane >> 4) == 0) a.r1[((size_t)c * a.K + l) * a.S_pad + s] = (cf.nw > 0.0) ? cf.nw * ratio : 0.0;
    }
    if (c >= a.n_tips) {
        if constexpr (NH || HESS) {
            // with Q from memory, or the Q^2 product as well, the fragments
            // load only now (held through the products they would spill)
            __builtin_amdgcn_sched_barrier(0);
            frags_issue(frag_of(a, c, l, 1), lane, F);
        }
        V16 acc = u;
        apply3f(F, u, acc);
        (void)rescale(acc);
        vstore(static_cast<float*>(a.qv) + mvec_off(a, c, tile), lane, acc);
    }
}

// Work items of the pre-order walk: each child of each node of a level is
// one item (item 2i + w of a level is child w of the level's i-th node), so
// a level offers twice as many independent items as nodes and a wave holds
// one child's state at a time.  Items go round-robin over the waves.  The
// tip codes of the item two ahead are in flight during an item; its own
// vectors (q of the node, the own and the sibling message or tip-table row)
// are loaded when the previous item is done, and its F^T fragments load
// under its Q product.  (Loading the vectors a whole item ahead needs 48
// more registers per lane and spills at two waves per SIMD.)
struct PreItem {
    V16 q, mown, msib;
};

__device__ inline int item_child(int4 nd, int w) { return w ? nd.z : nd.y; }
__device__ inline int item_sibling(int4 nd, int w) { return w ? nd.y : nd.z; }

// tip codes of the item's own child (x) and sibling (y)
__device__ inline uint2 item_codes(const EvalArgs& a, int4 nd, int w, int s) {
    uint2 cd = {0u, 0u};
    const int c = item_child(nd, w), b = item_sibling(nd, w);
    if (c < a.n_tips) cd.x = a.codes[(size_t)c * a.S_pad + s];
    if (b < a.n_tips) cd.y = a.codes[(size_t)b * a.S_pad + s];
    return cd;
}

__device__ inline void item_issue(const EvalArgs& a, int4 nd, int w, uint2 cd, int l, int tile, int lane,
                                  PreItem& r) {
    if (nd.x != a.root) {
        vload(static_cast<const float*>(a.qv) + mvec_off(a, nd.x, tile), lane, r.q);
    } else {
        const int g = lane >> 4;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * mt + 4 * g + i;
                r.q.v[mt][i] = x < a.M ? (float)a.pi64[x] : 0.f;
            }
    }
    ChildLd co, cb;
    const int c = item_child(nd, w), b = item_sibling(nd, w);
    co.code = cd.x;
    cb.code = cd.y;
    if (c >= a.n_tips) vload(static_cast<const float*>(a.msg) + mvec_off(a, c, tile), lane, co.v);
    if (b >= a.n_tips) vload(static_cast<const float*>(a.msg) + mvec_off(a, b, tile), lane, cb.v);
    child_finish(a, c, l, lane, co, r.mown);
    child_finish(a, b, l, lane, cb, r.msib);
}

// NH: per-branch rate matrices; each child's Q (and Q^2) fragments are
// read from memory (one block per matrix) instead of the LDS copies.
template <bool HESS, bool NH>
__device__ inline void mfma_pre_body(const EvalArgs& a, int tile, int4* lds_sched) {
    constexpr int QF = 3 * 8 * 64;  // bf16x8 per matrix
    __shared__ bf16x8 qop[NH ? 1 : QF];
    __shared__ bf16x8 q2lds[HESS && !NH ? QF : 1];
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
    const bf16x8* q2src = static_cast<const bf16x8*>(a.Q2op);
    if constexpr (!NH) {
        for (int i = threadIdx.x; i < QF; i += blockDim.x) qop[i] = qsrc[i];
        if constexpr (HESS)
            for (int i = threadIdx.x; i < QF; i += blockDim.x) q2lds[i] = q2src[i];
    }
    stage_schedule(a, lds_sched);
    __syncthreads();
    for (int h = a.n_levels - 1; h >= 0; --h) {
        const int base = a.level_off[h];
        const int n_it = 2 * (a.level_off[h + 1] - base);
        int it = wv;
        if (it < n_it) {
            int4 nd = sched_at(a, lds_sched, base + it / 2);
            PreItem cur;
            item_issue(a, nd, it & 1, item_codes(a, nd, it & 1, s), l, tile, lane, cur);
            int it1 = it + MW;
            uint2 cd1 = {0u, 0u};
            if (it1 < n_it) cd1 = item_codes(a, sched_at(a, lds_sched, base + it1 / 2), it1 & 1, s);
            while (true) {
                const bool more = it1 < n_it;
                int4 nn = nd;
                if (more) nn = sched_at(a, lds_sched, base + it1 / 2);
                const int it2 = it1 + MW;
                uint2 cd2 = {0u, 0u};
                if (it2 < n_it) cd2 = item_codes(a, sched_at(a, lds_sched, base + it2 / 2), it2 & 1, s);
                const int c = item_child(nd, it & 1);
                Frags F;
                if constexpr (!NH && !HESS)
                    if (c >= a.n_tips) frags_issue(frag_of(a, c, l, 1), lane, F);
                __builtin_amdgcn_sched_barrier(0);
                V16 u;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) u.v[mt] = cur.q.v[mt] * cur.msib.v[mt];
                const bf16x8* qc = qop;
                const bf16x8* q2c = q2lds;
                if constexpr (NH) {
                    // c is the same in every lane: a scalar base address
                    const size_t mo = (size_t)__builtin_amdgcn_readfirstlane(a.branch_model[c]) * QF;
                    qc = qsrc + mo;
                    q2c = q2src + mo;
                }
                mfma_pre_child<HESS, NH>(a, c, l, tile, s, lane, cf, u, cur.mown, qc, q2c, F);
                if (!more) break;
                nd = nn;
                item_issue(a, nd, it1 & 1, cd1, l, tile, lane, cur);
                it = it1;
                it1 = it2;
                cd1 = cd2;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- entry points

__global__ void __launch_bounds__(256) mfma_pmat_kernel(EvalArgs a) { mfma_pmat_body(a, blockIdx.x); }

__global__ void __launch_bounds__(MF_THREADS) mfma_post_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    mfma_post_body(a, tile, lds_dyn);
}

template <bool HESS, bool NH>
__global__ void __launch_bounds__(MF_THREADS) mfma_pre_kernel(EvalArgs a) {
    extern __shared__ int4 lds_dyn[];
    const int tile = xcd_tile(blockIdx.x, a.n_tiles);
    if (tile >= a.n_tiles) return;
    mfma_pre_body<HESS, NH>(a, tile, lds_dyn);
}

// Batched entry points for continuous batching: map[blockIdx.x] = {request,
// block within the request}; a request keeps exactly the blocks, order and
// results it has alone (the traversal block is the tile itself).
__global__ void __launch_bounds__(256) mfma_pmat_batch(const EvalArgs* __restrict__ reqs,
                                                        const int2* __restrict__ map) {
    const int2 m = map[blockIdx.x];
    mfma_pmat_body(reqs[m.x], m.y);
}
__global__ void __launch_bounds__(MF_THREADS) mfma_post_batch(const EvalArgs* __restrict__ reqs,
                                                              const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    mfma_post_body(reqs[m.x], m.y, lds_dyn);
}
__global__ void __launch_bounds__(MF_THREADS) mfma_pre_batch(const EvalArgs* __restrict__ reqs,
                                                             const int2* __restrict__ map) {
    extern __shared__ int4 lds_dyn[];
    const int2 m = map[blockIdx.x];
    // by value: uniform loads into scalar registers (through the reference
    // the fields would be held in vector registers, which spill)
    const EvalArgs a = reqs[m.x];
    mfma_pre_body<false, false>(a, m.y, lds_dyn);
}

size_t mfma_post_lds_bytes(const EvalArgs& a) { return sched_lds_bytes(a); }
size_t mfma_pre_lds_bytes(const EvalArgs& a) { return sched_lds_bytes(a); }

hipError_t launch_mfma_pmat(const EvalArgs& a, hipStream_t st) {
    mfma_pmat_kernel<<<(a.blist ? a.n_blist : a.n_branches) * a.K, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mfma_post(const EvalArgs& a, hipStream_t st) {
    mfma_post_kernel<<<N_XCD * xcd_per(a.n_tiles), MF_THREADS, mfma_post_lds_bytes(a), st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mfma_pre(const EvalArgs& a, hipStream_t st, bool hess) {
    const dim3 grid(N_XCD * xcd_per(a.n_tiles)), block(MF_THREADS);
    const size_t lds = mfma_pre_lds_bytes(a);
    if (a.n_models > 0) {
        if (hess) mfma_pre_kernel<true, true><<<grid, block, lds, st>>>(a);
        else mfma_pre_kernel<false, true><<<grid, block, lds, st>>>(a);
    } else {
        if (hess) mfma_pre_kernel<true, false><<<grid, block, lds, st>>>(a);
        else mfma_pre_kernel<false, false><<<grid, block, lds, st>>>(a);
    }
    return hipGetLastError();
}

// pmat, post and pre of a serving batch (the caller launches the reduction)
hipError_t launch_mfma_batch(const BatchLaunch& b, hipStream_t st) {
    if (b.pmat_blocks > 0) mfma_pmat_batch<<<b.pmat_blocks, 256, 0, st>>>(b.reqs, b.pmat_map);
    mfma_post_batch<<<b.trav_blocks, MF_THREADS, b.post_lds, st>>>(b.reqs, b.trav_map);
    mfma_pre_batch<<<b.trav_blocks, MF_THREADS, b.pre_lds, st>>>(b.reqs, b.trav_map);
    return hipGetLastError();
}

}  // namespace pg
