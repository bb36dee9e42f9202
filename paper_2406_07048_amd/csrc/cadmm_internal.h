// Internal declarations shared by the host (ABI) and kernel translation units
// of the gfx950 ADMM collision-avoidance library. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace cadmm {

constexpr int kWave = 64;
constexpr int kMaxWavesPerGroup = 8;
#define CADMM_MAX_NU_DEV 8
// bounds active at once in one scenario's trajectory QP (slots of the bounded solver)
constexpr int kBoundSlots = 64;

// Everything a kernel needs, passed by value (kernel argument segment).
struct DevProblem {
    int dim, n_s, n_u, N, n_parts, n_scen, n_blocks, n_wg;
    int att_kind, n_att, nq, nc;      // nq pose coordinates, nc contribution floats
    int pos_idx[3], att_idx[3];
    float sigma, eps_prox, eps_pri, eps_dual;
    int max_sweeps;
    int max_part_faces, max_obs_faces;   // select the compiled pair-kernel variant
    // geometry (FP32)
    const float4* part_faces;    // [F_r] (a_x, a_y, a_z, b)
    const int* part_face_ptr;    // [P+1]
    const float* part_off;       // [P*3]
    const float4* obs_faces;     // [F_o] (c_x, c_y, c_z, d)
    const double* obs_d64;       // [F_o] face offsets d in FP64
    const float4* obs_dc;        // [F_o] rounding of the FP32 normals, c - (float)c (FP32; w unused)
    const int* obs_face_ptr;     // [M+1]
    // pair blocks and work lists
    const int4* blocks;          // [n_blocks] (scenario, part, obstacle, n_rows)
    const int* block_yoff;       // [n_blocks] float offset of the block in y
    const int4* bdesc;           // [n_blocks] (first robot face, first obstacle face, y offset,
                                 //  robot faces | obstacle faces << 8 | part << 16)
    const int4* wg_items;        // [n_wg] (scenario, block_begin, block_end, wg index within scenario)
    const int2* scen_wg;         // [n_scen] (first wg, end wg)
    // model and cost
    const float* A_dyn;          // [n_models][n_s*n_s]; model of (s, t): s*dyn_ss + t*dyn_ts
    const float* B_dyn;          // [n_models][n_s*n_u]
    const float* c_dyn;          // [n_models][n_s]
    int dyn_ts, dyn_ss;
    int model;                   // 0 linear models; 1 bicycle, 2 quadrotor (relinearised every iteration)
    double model_par[8];
    float* A_lin;                // model != 0: [n_scen][N][n_s*n_s] the linearisation of the current iterate
    float* B_lin;                // model != 0: [n_scen][N][n_s*n_u]
    const float* Q_s;            // [n_s*n_s]
    const float* Q_u;            // [n_u*n_u]
    const float* x_ref;          // [n_scen*(N+1)*n_s]
    const float* x0;             // [n_scen*n_s]
    // iterate
    float* x;                    // [n_scen*(N+1)*n_s]
    float* u;                    // [n_scen*N*n_u]
    float* y;                    // canonical layout
    float* zeta;                 // [n_blocks*N]
    float* xi;                   // [n_blocks*dim*N]
    // per-iteration scratch
    float* contrib;              // [n_wg][nc][64]
    float* rdual_part;           // [n_wg]
    float* rpri_part;            // [n_wg]
    int* unconv_part;            // [n_wg]
    float* r_pri;                // [n_scen]
    float* r_dual;               // [n_scen]
    int* done;                   // [n_scen]
    int* iters;                  // [n_scen]
    int* unconv;                 // [n_scen]
    float* hist_pri;             // [hist_cap*n_scen]
    float* hist_dual;            // [hist_cap*n_scen]
    int hist_cap;
    // state and input bounds (has_bounds != 0): limits [n_s] / [n_u] (+-inf: none)
    int has_bounds;
    const float* xlo;
    const float* xhi;
    const float* ulo;
    const float* uhi;
    float* hq_b;                 // [n_scen][N][nc] stage sums of the last trajectory QP
    float* bW;                   // [2 n_scen][kBoundSlots][N (n_s + n_u)] active-bound directions, then
                                 // the precomputed directions of the previous active sets
    int* bprev;                  // [n_scen][kBoundSlots + 1] the previous active set (count, bound ids)
    // per-step sums of the pair contributions formed by a separate kernel
    // (scenarios with many pair-phase workgroups), [n_scen][N][nc]; NULL: the
    // trajectory kernel sums them itself
    const float* hq_pre;
    int* bstat;                  // [n_scen] active bounds, or < 0 (see traj_bounds_kernel)
};

// Inputs and outputs of the trajectory kernel in reverse mode (one adjoint LQ
// per scenario; see the trajectory kernel).
struct TrajAdjoint {
    const float* hq;       // [n_scen][N][nc] stage sums saved by the forward pass; NULL = obstacle-free
    const float* qpart;    // [n_wg][nq][64] pose cotangents per workgroup; NULL = none
    const float* xK;       // [n_scen][N+1][n_s] last trajectory for the cost gradient; NULL = none
    const float* uK;       // [n_scen][N][n_u] last inputs for the cost gradient; NULL = none
    float* w;              // [n_scen][N][n_s] out: w_t, t = 1..N
    double* gx0;           // [n_scen][n_s] accumulated cotangent of x_0
};

// Inputs and outputs of the reverse pair kernel for the step k -> k+1 of the
// iteration (all canonical layouts; see the reverse pair kernel).
struct PairAdjoint {
    const float* xk;       // trajectory x^k (poses of the pair QPs and stage terms)
    const float* xn;       // trajectory x^{k+1}
    const float* yk;       // duals y^k (proximal centre; multipliers of step k-1)
    const float* yn;       // duals y^{k+1}
    const float* zk;       // zeta^k
    const float* xik;      // xi^k
    const float* w;        // [n_scen][N][n_s] adjoint LQ trajectory of step k
    float* yb;             // in: cotangent of y^{k+1}; out: of y^k
    float* zb;             // in: of zeta^{k+1}; out: of zeta^k
    float* xib;            // in: of xi^{k+1}; out: of xi^k
    float* qpart;          // out: [n_wg][nq][64] pose cotangents of x^k per workgroup
    double* gdb;           // [n_parts][F_o] accumulated offset cotangents
    int n_obs_faces;       // F_o (row stride of gdb)
    int has_mult;          // k >= 1: include the multiplier update of step k-1
};

// Kernel launchers (defined in cadmm_kernels.hip / cadmm_adjoint.hip). All
// return hipError_t of the launch.
// Pair phase with W pair blocks per workgroup and G lanes per pair (1, 2, 4);
// a block takes ceil(N / (64 / G)) waves, and W times that must be <= 8.
// Launches of the ADMM phases. Given a pair of events (ev0 != nullptr), the
// launch records them around the kernel's own execution (hipExtLaunchKernel),
// which is what the per-phase timings use; graphs capture plain launches.
#define CADMM_LAUNCH(kernel, grid, block, lds, stream, ev0, ev1, ...)                                 \
    do {                                                                                           \
        if (ev0 || ev1) hipExtLaunchKernelGGL(kernel, grid, block, lds, stream, ev0, ev1, 0, __VA_ARGS__); \
        else hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                     \
    } while (0)

hipError_t launch_pair_phase(const DevProblem& P, int waves_per_group, int lanes_per_pair, int grid, hipStream_t s,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
bool pair_group_supported(int N, int W, int G);
hipError_t launch_mult_phase(const DevProblem& P, int waves_per_group, int grid, hipStream_t s,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_traj_phase(const DevProblem& P, int obstacle_free, hipStream_t s, float* hq_save = nullptr,
                             hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_traj_adjoint(const DevProblem& P, const TrajAdjoint& TA, hipStream_t s);
// Bounded trajectory QP after the trajectory kernel (P.has_bounds); ev1, if
// given, is recorded at the end of the kernel's execution.
hipError_t launch_traj_bounds(const DevProblem& P, int obstacle_free, hipStream_t s, hipEvent_t ev1 = nullptr);
bool bounds_supported(int n_s, int n_u);
hipError_t launch_pair_adjoint(const DevProblem& P, const PairAdjoint& A, int waves_per_group, int grid,
                               hipStream_t s);
hipError_t launch_grad_finalize(int n_parts, int n_faces, const double* gdb, int n_x0, const double* gx0,
                                float scale, float* grad_d, float* grad_x0, hipStream_t s);
hipError_t launch_residual(const DevProblem& P, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_init_pairs(const DevProblem& P, float* alpha_out, int write_y, hipStream_t s);
hipError_t launch_fill(float* p, long long n, float v, hipStream_t s);
hipError_t launch_set_face_offsets(float4* faces, const double* d64, int n, hipStream_t s);
hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t s);
hipError_t launch_cost(const DevProblem& P, float* cost_out, hipStream_t s);
hipError_t launch_min_alpha(const DevProblem& P, const float* alpha, float* out, hipStream_t s);

// Stateless pair-QP batch by the dual Newton method; with work (a counter and
// a queue, pair_qp_batch_work_bytes) in two launches: the second resumes the
// solves still running after a few sweeps.
hipError_t launch_pair_qp_batch(int n_pairs, int dim, const int* row_ptr, const float* K,
                                const float* kappa, const float* yhat, const float* bhat,
                                float eps, int max_sweeps, float* y, float* r, float* nu, int* status,
                                hipStream_t s, void* work = nullptr);
size_t pair_qp_batch_work_bytes(int n_pairs);
// The library's static buffer of the two-launch form on the current device
// (nullptr if its address cannot be found) and the pairs it holds.
void* noalloc_scratch();
int noalloc_max_pairs();
hipError_t launch_pair_qp_lemke(int n_pairs, int dim, const int* row_ptr, const float* K, const float* kappa,
                                const float* yhat, const float* bhat, float eps, int max_pivots, float* y, float* r,
                                float* nu, int* status, hipStream_t s);
hipError_t launch_scale_batch(int n_pairs, int dim, const int* a_ptr, const float* A, const float* b,
                              const int* o_ptr, const float* Cp, const float* dp, float* alpha,
                              float* lam, float* mu, int* status, hipStream_t s);

// Geometry limits of the compiled pair-kernel variants.
bool pair_variant_supported(int dim, int max_part_faces, int max_obs_faces);

}  // namespace cadmm
