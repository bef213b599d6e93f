// Internal declarations shared by the host (context, checks, schedule) and
// the device (kernels) translation units of libphylograd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/phylograd.h"

namespace pg {

// Patterns per tile: one tile is TP consecutive patterns of one rate
// category; 16 doubles (or floats) per state form one 128 B (64 B) run.
constexpr int TP = 16;
// Threads per workgroup of the traversal kernels: NS node slots x TP lanes.
constexpr int WG = 256;
constexpr int NS = WG / TP;

// Everything a kernel of one evaluation needs, passed by value.
struct EvalArgs {
    int n_tips, n_nodes, n_branches, root;
    int K, M, S, S_pad, n_pb, n_tiles, n_levels;
    double qnorm;                      // max_x sum_y |Q[x][y]|
    const double* t;                   // [B] branch lengths
    void* P;                           // [B][K][M][M] storage type
    void* msg;                         // [N-1][K][M][S_pad] outgoing messages P_k p_k
    void* qv;                          // [N-1][K][M][S_pad] pre-order vectors q_k
    const uint8_t* codes;              // [N][S_pad] tip codes
    const unsigned long long* masks;   // [256] code -> state mask
    const int* level_off;              // [H+1] offsets into level_nodes
    const int* level_nodes;            // internal nodes grouped by height
    const int2* children;              // [2N-1] children of internal nodes
    const double* Q64;                 // [M][M]
    const double* Q2_64;               // [M][M] Q*Q
    const double* pi64;                // [M]
    const double* rates;               // [K]
    const double* catw;                // [K]
    const double* weights;             // [S_pad], 0 on padding
    double* rootL;                     // [K][S_pad] pi^T p~_root per category
    int* rootE;                        // [K][S_pad] summed scale exponents
    double* rho;                       // [K][S_pad] posterior category weights
    double* partial;                   // [n_tiles][B] tile gradient sums
    double* partial2;                  // [n_pb][B] tile Hessian sums
    double* grad;                      // [B]
    double* hess;                      // [B]
    double* logL;                      // [1]
    int* status;                       // [1] 0 ok, 1 bad t, 2 zero likelihood
};

enum Precision { FP64 = PG_FP64, FP32 = PG_FP32 };

// Kernel launchers (kernels.hip).  Each returns a hipError_t from the launch.
bool kernel_supported(int M, int precision);
hipError_t launch_pmat(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_post(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_root(const EvalArgs& a, hipStream_t s);
hipError_t launch_pre(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_gsum(const EvalArgs& a, hipStream_t s);
hipError_t launch_hess(const EvalArgs& a, int precision, hipStream_t s);
hipError_t launch_hsum(const EvalArgs& a, hipStream_t s);

}  // namespace pg
