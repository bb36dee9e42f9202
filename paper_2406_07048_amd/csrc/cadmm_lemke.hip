// gfx950 kernel of the paper's own route for the dual-update QP (arXiv
// 2406.07048, Sec. IV-C), offered by the stateless batch entry point as the
// alternative to the dual Newton solver:
//   (1) one equality variable y_e (the largest kappa_e = b_k) is eliminated,
//       y_e = (1 - kappa_u^T y_u) / kappa_e, and its sign condition becomes
//       kappa~^T y_u <= eta~ (eq. const_least_square_ineq);
//   (2) the KKT conditions of that QP are the LCP w = M z + q, w, z >= 0,
//       w^T z = 0 with z = (y_u, phi) (eq. kkt_conditions and eq.
//       linear_complementarity_problem), the proximal term carried through
//       the elimination into M and q;
//   (3) Lemke's complementary pivoting solves the LCP.
// One wavefront per pair: lane i owns row i of the tableau [I | -M | -e | q]
// in LDS, the ratio test is a wave-wide arg-min and a pivot is one pass of
// each lane over its row. The LCP is solved in the variables scaled by the
// proximal metric (z'_u = sqrt(D_u) z_u; an LCP keeps its solutions under
// positive diagonal scaling, M' = S M S, q' = S q), which keeps the pivots'
// FP32 rounding on the scale of the rows.
#include "cadmm.h"
#include "cadmm_device.h"

#include <float.h>
#include <math.h>

namespace cadmm {

constexpr int kLemkeMaxRows = CADMM_MAX_PART_FACES + CADMM_MAX_OBS_FACES + 1;   // 41 rows of y
constexpr int kLemkeStride = 2 * kLemkeMaxRows + 2;                              // w, z, z0, rhs
// one wave (one pair) per workgroup: the pivot loops of different pairs run
// for different counts, so a workgroup barrier inside them could only be
// shared by a single wave
constexpr int kLemkeWaves = 1;

// arg-min of v over the wave (ties to the smaller key); lanes with
// v = +inf take no part. Every lane gets (v, key) of the winner.
__device__ __forceinline__ void wave_argmin(float& v, int& key)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float ov = __shfl_xor(v, o, 64);
        const int ok = __shfl_xor(key, o, 64);
        if (ov < v || (ov == v && ok < key)) { v = ov; key = ok; }
    }
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <int DIM>
__global__ void __launch_bounds__(64 * kLemkeWaves) pair_qp_lemke_kernel(int n_pairs, const int* row_ptr,
                                                                         const float* K, const float* kappa,
                                                                         const float* yhat, const float* bhat,
                                                                         float eps, int max_pivots, float* y,
                                                                         float* r, float* nu_out, int* status)
{
    constexpr int C = DIM + 1;
    __shared__ float T_all[kLemkeWaves][kLemkeMaxRows * kLemkeStride];
    __shared__ float Kt_all[kLemkeWaves][kLemkeMaxRows * C];
    __shared__ float ks_all[kLemkeWaves][kLemkeMaxRows];   // kappa~_u s_u
    __shared__ float kt_all[kLemkeWaves][kLemkeMaxRows];   // kappa~_u
    __shared__ float su_all[kLemkeWaves][kLemkeMaxRows];   // s_u
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = blockIdx.x * kLemkeWaves + wave;
    if (p >= n_pairs) return;                       // whole waves leave together
    float* T = T_all[wave];
    float* Kt = Kt_all[wave];
    float* ksl = ks_all[wave];
    float* ktl = kt_all[wave];
    float* sul = su_all[wave];
    const int r0 = row_ptr[p], n = row_ptr[p + 1] - r0;
    if (n < 2 || n > kLemkeMaxRows) {                // outside the tableau's size
        if (lane == 0) status[p] = -3;
        return;
    }
    const int m = n - 1;                            // y_u
    const int S = 2 * n + 2;                        // row length of the tableau
    const int cz0 = 2 * n, crhs = 2 * n + 1;
    // ---- rows of the pair, the eliminated row e, the scaled reduced rows ----
    float Kl[C] = {}, kl = 0.f, yhl = 0.f, Dl = 0.f;
    if (lane < n) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Kl[c] = K[(size_t)(r0 + lane) * C + c];
            Dl += Kl[c] * Kl[c];
        }
        kl = kappa[r0 + lane];
        yhl = yhat[r0 + lane];
    }
    float bh[C];
#pragma unroll
    for (int c = 0; c < C; ++c) bh[c] = bhat[(size_t)p * C + c];
    float kv = lane < n && kl > 0.f ? -kl : FLT_MAX;   // largest kappa first
    int e = lane;
    wave_argmin(kv, e);
    const float ke = __shfl(kl, e, 64), De = __shfl(Dl, e, 64), yhe = __shfl(yhl, e, 64);
    float Ke[C];
#pragma unroll
    for (int c = 0; c < C; ++c) Ke[c] = __shfl(Kl[c], e, 64);
    const float etat = 1.f / ke;
    // row u of the reduced problem is row l = u (u < e) or u + 1 (u >= e) of y
    const int l_of_u = lane < e ? lane : lane + 1;
    const bool urow = lane < m;
    float Ku[C] = {}, ku = 0.f, yhu = 0.f, Du = 1.f;
#pragma unroll
    for (int c = 0; c < C; ++c) Ku[c] = __shfl(Kl[c], l_of_u < 64 ? l_of_u : 0, 64);
    ku = __shfl(kl, l_of_u < 64 ? l_of_u : 0, 64);
    yhu = __shfl(yhl, l_of_u < 64 ? l_of_u : 0, 64);
    Du = __shfl(Dl, l_of_u < 64 ? l_of_u : 0, 64);
    const float kt = urow ? ku / ke : 0.f;          // kappa~_u
    const float su = urow ? __builtin_amdgcn_rsqf(fmaxf(Du, 1e-30f)) : 1.f;   // scale of z_u
    float bt[C];
#pragma unroll
    for (int c = 0; c < C; ++c) bt[c] = bh[c] + Ke[c] * etat;
    if (urow) {
#pragma unroll
        for (int c = 0; c < C; ++c) Kt[lane * C + c] = Ku[c] - kt * Ke[c];
        ksl[lane] = kt * su;
        ktl[lane] = kt;
        sul[lane] = su;
    }
    __syncthreads();
    // ---- tableau row i = lane: [I | -M' | -1 | q'] ----
    if (lane < n) {
        float* Ti = T + lane * S;
        for (int j = 0; j < S; ++j) Ti[j] = 0.f;
        Ti[lane] = 1.f;
        Ti[cz0] = -1.f;
        if (urow) {
            float Ktu[C], cu = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) { Ktu[c] = Kt[lane * C + c]; cu += Ktu[c] * bt[c]; }
            // gradient at y_u = 0 (y_e = eta~) with the proximal term
            cu += eps * (-kt * De * (etat - yhe) - Du * yhu);
            for (int v = 0; v < m; ++v) {
                const float kv2 = ktl[v], sv = sul[v];
                float q = 0.f;
#pragma unroll
                for (int c = 0; c < C; ++c) q += Ktu[c] * Kt[v * C + c];
                q += eps * De * kt * kv2;
                if (v == lane) q += eps * Du;
                Ti[n + v] = -su * q * sv;
            }
            Ti[n + m] = -su * kt;                   // s_phi = 1
            Ti[crhs] = su * cu;
        } else {
            // the phi row: w_phi = eta~ - kappa~^T y_u
            for (int v = 0; v < m; ++v) Ti[n + v] = ksl[v];
            Ti[crhs] = etat;
        }
    }
    __syncthreads();
    // ---- Lemke's method ----
    int basis = lane;                                // w_i basic in row i
    float qv = lane < n ? T[lane * S + crhs] : FLT_MAX;
    int leave = lane;
    wave_argmin(qv, leave);
    int piv = 0, st = 0;
    if (qv < 0.f) {
        int enter = cz0;
        for (;;) {
            if (piv >= max_pivots) { st = -2; break; }
            ++piv;
            const float pr = T[leave * S + enter];
            const float ipr = 1.f / pr;
            if (lane < n) {
                float* Ti = T + lane * S;
                const float* Tl = T + leave * S;
                const float f = lane == leave ? 0.f : Ti[enter] * ipr;
                for (int j = 0; j < S; ++j) {
                    const float tl = Tl[j];
                    Ti[j] = lane == leave ? tl * ipr : Ti[j] - f * tl;
                }
            }
            __syncthreads();
            const int left = __shfl(basis, leave, 64);
            if (lane == leave) basis = enter;
            if (left == cz0) break;                  // z0 left the basis: solved
            enter = left < n ? n + left : left - n;  // the complement of the leaving variable
            // minimum ratio over rows with a positive entry in the entering column
            const float a = lane < n ? T[lane * S + enter] : 0.f;
            const float amax = wave_max(fabsf(a));
            float ratio = FLT_MAX;
            if (lane < n && a > 1e-6f * amax) ratio = T[lane * S + crhs] / a;
            int row = lane;
            wave_argmin(ratio, row);
            if (ratio == FLT_MAX) { st = -1; break; } // secondary ray
            leave = row;
        }
    }
    // ---- solution: z_u = s_u z'_u, y_e from the equality ----
    float zu = 0.f;
    {
        // row i holds basic variable basis(i) with value rhs(i)
        const float rhs = lane < n ? T[lane * S + crhs] : 0.f;
        for (int i = 0; i < n; ++i) {
            const int bi = __shfl(basis, i, 64);
            const float vi = __shfl(rhs, i, 64);
            if (bi >= n && bi < 2 * n && bi - n == lane) zu = fmaxf(vi, 0.f);
        }
    }
    const float yu = urow ? su * zu : 0.f;
    const float ye = etat - wave_sum(urow ? kt * yu : 0.f);
    // y in row order: lane l < n takes y_u of its reduced index, or y_e
    const int u_of_l = lane < e ? lane : lane - 1;
    const float yfrom = __shfl(yu, u_of_l >= 0 && u_of_l < 64 ? u_of_l : 0, 64);
    const float yl = lane == e ? fmaxf(ye, 0.f) : (lane < n ? yfrom : 0.f);
    if (lane < n) y[r0 + lane] = yl;
    float rr[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rr[c] = bh[c] + wave_sum(lane < n ? yl * Kl[c] : 0.f);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) r[(size_t)p * C + c] = rr[c];
    }
    // the multiplier of kappa^T y = 1 from the stationarity of the lambda row
    // with the largest kappa_l y_l (its w_l is zero)
    float kyv = lane < n && kl > 0.f ? -kl * yl : FLT_MAX;
    int lk = lane;
    wave_argmin(kyv, lk);
    float Kr = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) Kr += Kl[c] * rr[c];
    const float nl = (Kr + eps * Dl * (yl - yhl)) / (kl > 0.f ? kl : 1.f);
    const float nu = __shfl(nl, lk, 64);
    if (lane == 0) {
        nu_out[p] = nu;
        status[p] = st < 0 ? st : piv;
    }
}

hipError_t launch_pair_qp_lemke(int n_pairs, int dim, const int* row_ptr, const float* K, const float* kappa,
                                const float* yhat, const float* bhat, float eps, int max_pivots, float* y,
                                float* r, float* nu, int* status, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (n_pairs + kLemkeWaves - 1) / kLemkeWaves;
    if (dim == 2)
        hipLaunchKernelGGL(pair_qp_lemke_kernel<2>, dim3(grid), dim3(64 * kLemkeWaves), 0, st, n_pairs, row_ptr, K,
                           kappa, yhat, bhat, eps, max_pivots, y, r, nu, status);
    else
        hipLaunchKernelGGL(pair_qp_lemke_kernel<3>, dim3(grid), dim3(64 * kLemkeWaves), 0, st, n_pairs, row_ptr, K,
                           kappa, yhat, bhat, eps, max_pivots, y, r, nu, status);
    return hipGetLastError();
}

}  // namespace cadmm
