// Internal declarations shared by the host (context, checks, schedule) and
// the device (kernels) translation units of libphylograd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/phylograd.h"
#include "plan.h"

namespace pg {

// Node slots per workgroup of the traversal kernels (each slot is TP lanes):
// the workgroup has node_slots(M) * TP threads.
__host__ __device__ constexpr int node_slots(int M) { return M <= 8 ? 32 : 16; }
// Branches per block of the gradient reduction.
constexpr int GS_BRANCHES = 16;
// Wavefronts (clade lists) per workgroup of the separate clade launches.
constexpr int CW_WAVES = 4;
// Node slots of the pre-order kernel (FP64 small M: fewer, heavier slots).
#ifndef PG_PRE_NS64
#define PG_PRE_NS64 16
#endif
#ifndef PG_PRE_WPE64
#define PG_PRE_WPE64 1
#endif
template <typename T>
__host__ __device__ constexpr int pre_slots(int M) {
    return (M * M <= TP && sizeof(T) == 8) ? PG_PRE_NS64 : node_slots(M);
}
template <typename T>
__host__ __device__ constexpr int pre_waves(int M) {
    return M * M <= TP ? (sizeof(T) == 8 ? PG_PRE_WPE64 : 4) : 1;
}
inline int pre_node_slots(int M, int precision) {
    return precision == PG_FP32 ? pre_slots<float>(M) : pre_slots<double>(M);
}
// Node slots of the post-order kernel: as many as the pre-order kernel's for
// small M, so both walk the same clade lists (the pre-order walk then reads
// first the messages the post-order walk wrote last, while still cached).
template <typename T>
__host__ __device__ constexpr int post_slots(int M) {
    return M * M <= TP ? pre_slots<T>(M) : node_slots(M);
}
inline int post_node_slots(int M, int precision) {
    return precision == PG_FP32 ? post_slots<float>(M) : post_slots<double>(M);
}
__host__ __device__ inline int gsum_blocks(int n_branches) {
    return (n_branches + GS_BRANCHES - 1) / GS_BRANCHES;
}

// Everything a kernel of one evaluation needs, passed by value.
struct EvalArgs {
    int n_tips, n_nodes, n_branches, root;
    int K, M, S, S_pad, n_pb, n_tiles, n_levels;
    double qnorm;                      // max_x sum_y |Q[x][y]|
    double Qs[16];                     // Q by value when M*M <= 16 (kernel arguments
    double pis[4];                     // are uniform: read through the scalar cache)
    double Q2s[16];                    // Q*Q by value when M*M <= 16
    const double* t;                   // [B] branch lengths (device)
    void* P;                           // [B][K][M][M] storage type
    void* msg;                         // [N-1][n_tiles][M][TP] outgoing messages P_k p~_k
    void* qv;                          // [N-1][n_tiles][M][TP] pre-order vectors q~_k
    const uint8_t* codes;              // [N][S_pad] tip codes
    const unsigned long long* masks;   // [256] code -> state mask
    const int* level_off;              // [H+1] offsets into sched, by level
    const int4* sched;                 // [N-1] {node, child 0, child 1, 0}, internal
                                       //       nodes grouped by height
    int sched_lds;                     // 1: traversal kernels stage sched in LDS
    int top_level;                     // first level of the pre-order top region
                                       // (n_levels: none)
    int top_nodes;                     // nodes in the top region (LDS blocks)
    int n_sched;                       // entries of sched (the top nodes when
                                       // clades are walked, else all N-1)
    // clade walks: entries {node, first child, second child, CL_* flags} in
    // post order within each clade (the child with more internal nodes
    // first), clades grouped by node slot; the pre-order kernel walks its
    // list backwards.  The two kernels' lists differ when their slot counts do.
    int n_cl;                          // entries per list (0: no clades)
    int cl_depth;                      // stack blocks (M x TP) per node slot
    const int4* cl_post;               // [n_cl]
    const int* cl_post_off;            // [post slots + 1] slot ranges
    const int4* cl_pre;                // [n_cl]
    const int* cl_pre_off;             // [pre slots + 1]
    int* cl_esum;                      // [post slots / 4][n_tiles][TP] exponent sums of the
                                       //   clade launch (NULL: clades walked inside the
                                       //   traversal kernels)
    int n_cl_esum;                     // parts of cl_esum the top-level launch adds
    const double* Q64;                 // [M][M]
    const double* Q2_64;               // [M][M] Q*Q
    const double* pi64;                // [M]
    const double* rates;               // [K]
    const double* catw;                // [K]
    const double* weights;             // [S_pad], 0 on padding
    double* rootL;                     // [K][S_pad] pi^T p~_root per category
    int* rootE;                        // [K][S_pad] summed scale exponents
    double* partial;                   // [n_tiles][B] tile gradient sums
    double* logl_part;                 // [n_pb] sum_s w_s log L_s of each pattern block
    int* flag_part;                    // [n_pb] 1 NaN, 2 zero likelihood in the block
    double* partial2;                  // [n_tiles][B] tile sums of the Hessian's additive part
    double* r1;                        // [B][K][S_pad] per-site gradient parts (Hessian)
    double* grad_out;                  // [B] gradient destination
    double* hess_out;                  // [B] Hessian-diagonal destination
    double* logL_out;                  // [1] logL destination
    int* status;                       // [1] written by each logL reduction: 0 ok,
                                       //     1 NaN (bad length), 2 zero likelihood
    // non-homogeneous model (n_models > 0): branch b uses rate matrix
    // Qm[branch_model[b]] instead of Q64 / Qs
    int n_models;
    const int* branch_model;           // [B]
    const double* Qm;                  // [n_models][M][M]
    const double* Q2m;                 // [n_models][M][M] squares
    const double* qnorm_m;             // [n_models] max row abs sum
    // partial re-evaluation: pmat over a branch list, per-node scale
    // exponents kept so a post-order pass over some nodes can patch rootE
    const int* blist;                  // [n_blist] branches whose P to form (NULL: all)
    int n_blist;
    int16_t* expo;                     // [N-1][n_tiles][TP] exponent of each node (NULL: off)
    int expo_delta;                    // 1: this post-order pass visits only some nodes;
                                       //    rootE += sum of (new - stored) exponents
    // split-BF16 path: states padded to MP, P holds per-(branch, category)
    // operand slots of MF_SLOT_BYTES, msg/qv hold MP x TP FP32 per tile
    const double* eV;                  // [MP][MP] V of Q = V B V^-1, identity on padding
    const double* eVinv;               // [MP][MP]
    const double* eRe;                 // [MP] eigenvalue real parts
    const double* eIm;                 // [MP] imaginary parts of pairs
    const int* eKind;                  // [MP] 0 real, 1 / 2 the two columns of a pair
    int expm_taylor;                   // 1: scaling and squaring (Q not usably diagonalisable)
    const void* Qop;                   // Q as MFMA A operands, three BF16 parts
    const void* Q2op;                  // Q^2 likewise (Hessian)
    // dense-state path: A fragments of Q and Q^2 of each rate matrix
    // ([max(1, n_models)][2][DN_NF][64], the path's type)
    const void* Qfrag;
};

enum Precision { FP64 = PG_FP64, FP32 = PG_FP32, SPLIT_BF16 = PG_SPLIT_BF16 };

// Split-BF16 path: padded state count, bytes of one (branch, category)
// operand slot (A operands of P - I and P^T - I in three BF16 parts for an
// internal branch, the FP32 tip table of P for a tip branch), and bytes of
// Q's A operands.
constexpr int MP = 64;
constexpr size_t MF_SLOT_BYTES = 49152;
constexpr size_t MF_QOP_BYTES = 3 * 8 * 64 * 16;

// Dense-state path (FP64 / FP32 partials, 16 < M <= 32, e.g. 20 amino
// acids): products on the matrix cores (16 x 16 x 4 MFMA), a vector of M
// states x 16 patterns held as two 16-row blocks of the MFMA accumulator.
// The accumulator's lane L = 16 g + c holds column c and, in its register
// r, row 4 g + r (FP32) or g + 4 r (FP64): dn_b0_state.  Lane L holds
// pattern c: in row block 0 the states dn_b0_state(g, r) (r < 4), in row
// block 1 the states 16 + K1 g + r (r < K1, K1 = ceil((M - 16) / 4)); the
// other rows of block 1 are padding.  A product A x runs KS = 4 + K1
// k-steps per output block; at k-step s lane group k contributes the state
// dn_col_state(s, k), which is the lane's own register s (block 0) or
// s - 4 (block 1), so a product's output is the next product's input.  A
// matrix is stored as dn_nf(M) = 2 KS fragments per lane, [ob][s][lane]:
// entry A[dn_row_state(ob, L % 16)][dn_col_state(s, L / 16)] (0 for
// padding).  `wide` selects the FP64 register order.
constexpr bool dense_states(int M) { return M > 16 && M <= 32; }
constexpr int dn_k1(int M) { return (M - 16 + 3) / 4; }
constexpr int dn_ks(int M) { return 4 + dn_k1(M); }
constexpr int dn_nf(int M) { return 2 * dn_ks(M); }
// states as stored per pattern (M rounded up to a multiple of 4)
constexpr int dn_md(int M) { return 16 + 4 * dn_k1(M); }
constexpr int dn_b0_state(int g, int r, bool wide) { return wide ? g + 4 * r : 4 * g + r; }
constexpr int dn_row_state(int M, int ob, int i, bool wide) {
    // row i of block 1 is register r of lane group g
    return ob == 0 ? i
                   : ((wide ? i / 4 : i % 4) < dn_k1(M) &&
                              16 + dn_k1(M) * (wide ? i % 4 : i / 4) + (wide ? i / 4 : i % 4) < M
                          ? 16 + dn_k1(M) * (wide ? i % 4 : i / 4) + (wide ? i / 4 : i % 4)
                          : -1);
}
constexpr int dn_col_state(int M, int s, int k, bool wide) {
    return s < 4 ? dn_b0_state(k, s, wide)
                 : (16 + dn_k1(M) * k + (s - 4) < M ? 16 + dn_k1(M) * k + (s - 4) : -1);
}
// entries (of the path's type) of one (branch, category) transition-matrix
// slot: the fragments of P and of P^T (internal branch) or the tip table,
// rows y < M = column y of P and row M = P 1, MD entries each in the lanes'
// register order: entry 4 g + r is state dn_b0_state(g, r), entry 16 + j is
// state 16 + j (tip branch)
constexpr int dn_slot_elems(int M) {
    return 2 * dn_nf(M) * 64 > (M + 1) * dn_md(M) ? 2 * dn_nf(M) * 64 : (M + 1) * dn_md(M);
}
// Q fragments then Q^2 fragments, per rate matrix
constexpr int dn_qfrag_elems(int M) { return 2 * dn_nf(M) * 64; }

// Kernel launchers (kernels.hip).  Each returns a hipError_t from the launch.
bool kernel_supported(int M, int precision);
inline size_t sched_lds_bytes(const EvalArgs& a) { return a.sched_lds ? sizeof(int4) * a.n_sched : 0; }
inline size_t top_lds_bytes(const EvalArgs& a, size_t elem) { return elem * (size_t)a.top_nodes * a.M * TP; }
hipError_t launch_pmat(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_post(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_logl(const EvalArgs& a, hipStream_t s);
hipError_t launch_pre(const EvalArgs& a, int precision, hipStream_t s, bool hess);
hipError_t launch_hsum(const EvalArgs& a, hipStream_t s);
// split-BF16 launchers (kernels_mfma.hip)
hipError_t launch_mfma_pmat(const EvalArgs& a, hipStream_t s);
hipError_t launch_mfma_post(const EvalArgs& a, hipStream_t s);
hipError_t launch_mfma_pre(const EvalArgs& a, hipStream_t s, bool hess);
// dense-state launchers (kernels_dense.hip)
hipError_t launch_dense_pmat(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_dense_post(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_dense_pre(const EvalArgs& a, int precision, hipStream_t s, bool hess);
size_t mfma_post_lds_bytes(const EvalArgs& a);
size_t mfma_pre_lds_bytes(const EvalArgs& a);

// One continuous-batching step: every request's pmat, post, pre and gsum
// blocks in one launch each.  reqs and the maps are device arrays; map
// entries are {request index, block within the request}.
struct BatchLaunch {
    int M, precision;
    const EvalArgs* reqs;
    const EvalArgs* reqs_top;  // the traversal launches' arguments (clade_top_args), or NULL: reqs
    const int2* pmat_map;
    const int2* trav_map;
    const int2* gsum_map;
    const int2* clade_map;     // {request, block} of the clade launches
    int pmat_blocks, trav_blocks, gsum_blocks, clade_blocks;
    size_t post_lds, pre_lds, clade_lds;
    int top_kernels;   // 1: every request's top levels take the top-level launches (top_launch_ok)
    size_t top_lds;    // their dynamic LDS (largest top_launch_lds)
};
// Separate clade launches of small-M requests: their blocks (0: none), the
// arguments of their top-level (traversal) launches, their dynamic LDS.
int clade_blocks(const EvalArgs& a, int precision);
EvalArgs clade_top_args(const EvalArgs& a, int precision);
size_t clade_lds_bytes(const EvalArgs& a, int precision);
bool top_launch_ok(const EvalArgs& top, int precision);
size_t top_launch_lds(const EvalArgs& top, int precision);
int pmat_blocks(const EvalArgs& a, int precision);
int traversal_blocks(const EvalArgs& a);
int gsum_total_blocks(const EvalArgs& a);
size_t post_lds_bytes(const EvalArgs& a, int precision);
size_t pre_lds_bytes(const EvalArgs& a, int precision);
hipError_t launch_batch(const BatchLaunch& b, hipStream_t s);
hipError_t launch_dense_batch(const BatchLaunch& b, hipStream_t s);  // kernels_dense.hip
hipError_t launch_mfma_batch(const BatchLaunch& b, hipStream_t s);   // kernels_mfma.hip

// Q = V B V^-1 with B block diagonal (eigen.cpp).  kind[j]: 0 real
// eigenvalue re[j]; 1 and 2 the two columns (real and imaginary part of the
// eigenvector of re + i im) of a conjugate pair.  Row-major m x m.
struct EigenSystem {
    int m = 0;
    std::vector<double> V, Vinv, re, im;
    std::vector<int> kind;
    double cond = 0.0;   // ||V||_1 ||V^-1||_1
    double resid = 0.0;  // max |V B V^-1 - Q| / max |Q|
};
bool eigen_decompose(int m, const double* Q, EigenSystem& es);

// Device memory source of a context (the serving scheduler's pool).
// acquire returns a block of at least `bytes` (its size in *granted), or
// NULL; both calls may come from different threads.
struct DeviceAllocator {
    virtual void* acquire(size_t bytes, size_t* granted) = 0;
    virtual void release(void* p, size_t bytes) = 0;
    virtual ~DeviceAllocator() = default;
};

// Context internals used by the serving scheduler (capi.cpp).
}  // namespace pg
struct pg_ctx;
namespace pg {
pg_ctx* ctx_new_session(int device, int precision, hipStream_t stream, DeviceAllocator* alloc);
// Host planning of the device state (no device work).
int ctx_plan(pg_ctx* c);
// Device bytes the context's buffers take when each allocation is rounded
// up to a multiple of `granule`.
int64_t ctx_need_bytes(pg_ctx* c, size_t granule);
// Allocate and upload on `stream` (waits for it), then keep using the
// context's own stream.
int ctx_prepare(pg_ctx* c, hipStream_t stream);
EvalArgs ctx_args(const pg_ctx* c);
int ctx_precision(const pg_ctx* c);
const char* ctx_error(const pg_ctx* c);
hipError_t launch_gsum(const EvalArgs& a, hipStream_t s);


}  // namespace pg
