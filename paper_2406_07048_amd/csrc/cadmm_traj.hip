// gfx950 kernels of the trajectory-QP step of the ADMM collision-avoidance
// path (arXiv 2406.07048, Sec. IV-B state update): per-step sums of the pair
// contributions, the backward Riccati sweep and the forward rollout, in
// forward mode and as the adjoint LQ of the reverse pass.
#include "cadmm.h"
#include "cadmm_device.h"
#include "cadmm_model.h"

#include <float.h>
#include <math.h>

namespace cadmm {

// accumulator of a 16 x 16 x 4 FP32 matrix-core product (4 registers a lane)
typedef float v4f __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------
// ADMM step 2: trajectory QP by a backward Riccati sweep and forward
// rollout; one workgroup per scenario. The QP is solved in deviation
// coordinates about the current iterate, dx = x - x^k, du = u - u^k: stage
// cost 1/2 dx^T H_t dx + g_t^T dx with H_t = 2 Q_s + sum_ij sigma J^T J and
// g_t = 2 Q_s (x^k_t - xref_t) + sum_ij sigma J^T e (pose block), input cost
// 1/2 du^T (2 Q_u) du + (2 Q_u u^k_t)^T du, dynamics dx_{t+1} = A dx_t +
// B du_t + f_t with the defect f_t = A x^k_t + B u^k_t + c - x^k_{t+1} formed
// in FP64. This is the same QP as in absolute coordinates, without the
// cancellation of sigma J^T J q^k against the positions of the scene.
// The obstacle-free solve (initial iterate) uses the base point 0.
//
// Reverse mode (ADJ): the same sweep solves the adjoint LQ of one forward
// trajectory QP. With xbar_t, ubar_t the cotangents of its solution (x, u),
// the vector abar = Hs^{-1} (ubar + sum_t M_t^T xbar_t) of the condensed
// problem (Hs its input Hessian, M_t the input-to-state map) is the minimiser
// of the same LQ with h_t = -xbar_t, an input term -ubar_t, c = 0 and
// x_0 = 0, and its state trajectory w_t = M_t abar is what the stage
// adjoints need (Hbar_t = -(w_t x_t^T + x_t w_t^T) / 2, hbar_t = -w_t). The
// cotangent of x_0 is sum_t (A^T)^t (xbar_t - H_t w_t), accumulated by a
// Horner sweep after the rollout.
// ------------------------------------------------------------------------

// Threads of the trajectory kernel: enough for one output per thread in
// every phase of the LDS sweep (at most 400 for the 16/8 padding), and for
// the per-step sums to split each output's workgroup partials over several
// threads (C3: 270 outputs over 1024 threads). The 16/8 padding keeps 512,
// whose register budget holds its larger sweep without spills.
__host__ __device__ constexpr int traj_threads(int NS, int) { return NS > 12 ? 512 : 1024; }

// Floats of the gains region, which first holds the staged trajectory
// (x and x_ref over t = 0..N, u over t = 0..N-1, padded to NS / NU).
__host__ __device__ inline int traj_gain_floats(int N, int NS, int NU)
{
    const int gains = N * NU * (NS + 1), stage = 2 * (N + 1) * NS + N * NU;
    return gains > stage ? gains : stage;
}

// Dynamic LDS floats of the trajectory kernel for padded sizes NS, NU
// (reverse mode adds the w trajectory).
__host__ __device__ constexpr int al4(int n) { return (n + 3) & ~3; }

// The last region holds the chunk sums of the per-step sums (4 TT floats),
// and afterwards, for the closed-loop rollout (cl), A + B K_t and f_t + B k_t
// of every step (N NS (NS + 1) floats; at NS = 12 as 12 x 16 rows of the
// homogeneous maps, N 192 floats).
// Time-varying models on the register path (4/2) add the padded A_t, B_t of
// every step ([N][24] floats).
__host__ __device__ inline int traj_dyn_floats(int N, int NS, int NU, int nc, bool adj, bool cl, bool tv = false)
{
    const int clf = NS == 12 ? N * 12 * 16 : N * NS * (NS + 1);
    const int tail = cl && clf > 4 * traj_threads(NS, NU) ? clf : 4 * traj_threads(NS, NU);
    return al4(N * nc) + al4(N * NS) + al4(traj_gain_floats(N, NS, NU)) + al4(N * NU) + al4(N * NS) +
           (adj ? al4((N + 1) * NS) : 0) + (tv && NS == 4 ? al4(N * 24) : 0) + tail;
}

// ------------------------------------------------------------------------
// Nonlinear dynamics F(s, u) = s + dt f_c(s, u) (cadmm_model.h) and one
// column of its Jacobian, by forward-mode derivatives (a value and one
// tangent, FP64): one thread per (step, column). Column j < n_s is dF/ds_j,
// else dF/du_{j - n_s}.
// ------------------------------------------------------------------------
template <int MODEL>
__device__ __forceinline__ void model_column(int model, const double* par, const float* s, const float* u, int j,
                                             const ModelTrig& tr, double* F, double* col)
{
    // MODEL > 0: the model fixed at compile time (its sizes unrolled)
    const int ns = MODEL ? model_ns(MODEL) : model_ns(model), nu = MODEL ? model_nu(MODEL) : model_nu(model);
    if (MODEL) model = MODEL;
    Tan S[12], U[4], f[12];
    for (int i = 0; i < ns; ++i) S[i] = {(double)s[i], i == j ? 1.0 : 0.0};
    for (int k = 0; k < nu; ++k) U[k] = {(double)u[k], ns + k == j ? 1.0 : 0.0};
    model_fc<Tan>(model, par, S, U, f, &tr);
    const double dt = par[0];
    for (int i = 0; i < ns; ++i) {
        F[i] = (double)s[i] + dt * f[i].v;
        col[i] = (i == j ? 1.0 : 0.0) + dt * f[i].d;
    }
}

// Fixed-order sum of the float4 src[w * stride], w = w0..w1-1, with eight
// independent partial sums (w - w0 mod 8). Loads are issued sixteen at a
// time ahead of their use (the scheduling barrier keeps the compiler from
// interleaving each load with its add, which serialises the L2 round trips).
__device__ __forceinline__ float4 strided_sum4(const float4* src, size_t stride, int w0, int w1)
{
    float4 a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    int w = w0;
    for (; w + 16 <= w1; w += 16) {
        float4 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = src[(size_t)(w + q) * stride];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            a[q & 7].x += v[q].x; a[q & 7].y += v[q].y; a[q & 7].z += v[q].z; a[q & 7].w += v[q].w;
        }
    }
    if (w + 8 <= w1) {
        float4 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[(size_t)(w + q) * stride];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            a[q].x += v[q].x; a[q].y += v[q].y; a[q].z += v[q].z; a[q].w += v[q].w;
        }
        w += 8;
    }
    {
        float4 v[7];
#pragma unroll
        for (int q = 0; q < 7; ++q)
            v[q] = w + q < w1 ? src[(size_t)(w + q) * stride] : make_float4(0.f, 0.f, 0.f, 0.f);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 7; ++q)
            if (w + q < w1) {
                a[q].x += v[q].x; a[q].y += v[q].y; a[q].z += v[q].z; a[q].w += v[q].w;
            }
    }
    float4 r;
    r.x = ((a[0].x + a[1].x) + (a[2].x + a[3].x)) + ((a[4].x + a[5].x) + (a[6].x + a[7].x));
    r.y = ((a[0].y + a[1].y) + (a[2].y + a[3].y)) + ((a[4].y + a[5].y) + (a[6].y + a[7].y));
    r.z = ((a[0].z + a[1].z) + (a[2].z + a[3].z)) + ((a[4].z + a[5].z) + (a[6].z + a[7].z));
    r.w = ((a[0].w + a[1].w) + (a[2].w + a[3].w)) + ((a[4].w + a[5].w) + (a[6].w + a[7].w));
    return r;
}

// Fixed-order sums over the workgroup partials [w0, w1) for O float4
// outputs (src(o): the float4 of output o in workgroup w0, stride between
// workgroups). With TT >= 2 O threads each output's workgroups are split
// into S <= 8 contiguous chunks, summed by S threads and combined in chunk
// order through red4 (TT float4 of LDS); out(o, v) receives the sums.
// Every thread of the block calls it (it may hold a barrier).
template <int TT, class Src, class Out>
__device__ __forceinline__ void split_sums(int O, int w0, int w1, size_t stride, float4* red4, Src src, Out out)
{
    const int tid = threadIdx.x;
    const int S = O > 0 ? max(1, min(8, TT / O)) : 1;
    if (S == 1) {
        for (int o = tid; o < O; o += TT) out(o, strided_sum4(src(o), stride, w0, w1));
        return;
    }
    const int chunk = (w1 - w0 + S - 1) / S;
    if (tid < O * S) {
        const int o = tid % O, k = tid / O;
        const int a = w0 + k * chunk, b = min(w1, a + chunk);
        red4[tid] = a < b ? strided_sum4(src(o), stride, a, b) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    if (tid < O) {
        float4 v = red4[tid];
        for (int k = 1; k < S; ++k) {
            const float4 u = red4[k * O + tid];
            v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
        }
        out(tid, v);
    }
}

// acc + x . y for two 16-byte aligned NS-vectors in LDS (NS a multiple of 4),
// summed in index order, read as float4.
template <int NS>
__device__ __forceinline__ float dot_lds(const float* x, const float* y, float acc)
{
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
#pragma unroll
    for (int q = 0; q < NS / 4; ++q) {
        const float4 a = x4[q], b = y4[q];
        acc += a.x * b.x;
        acc += a.y * b.y;
        acc += a.z * b.z;
        acc += a.w * b.w;
    }
    return acc;
}

// Riccati sweep for 4 states and 2 inputs in one wave on 16 x 16 x 4 FP32
// matrix-core tiles (the layouts and the step of riccati_mfma_124), with the
// variables embedded so that every product needs one or two K-slices: the
// states at tile indices 0, 4, 8, 12 (slice 0 of lane rows 0-3), input 0 at
// 1, the affine 1 at 2 and input 1 at 3 (slices 1, 2, 3 of lane row 0).
//   W  = P^T M                     slice 0            (1 product)
//   Z1 = blkdiag(H_t, 2Q_u) + M^T W slice 0            (1)
//   Z2 = H_t, (h_t; r_t) + W^T [M | f^]  slices 0 and 2 (2: row 2 of W is p^T M)
//   P^_t = [Qxx qx] + Qux^T [K | k]  slices 1 and 3    (2)
// Qux columns and qu then sit in lane row 0 (registers 1 and 3), so the
// gains of column c are formed in lane c with the 2 x 2 inverse of Quu (three
// readlanes); 1/2 (Z1 + Z2) is exactly symmetric as in the 12-state sweep.
// Gains go to Kall[t][2][5] for rollout_scan_42; with TV the model of step t
// is A + t mstride, B + t mstride (padded 4 x 4 and 4 x 2, in LDS).
template <bool ADJ, bool TV>
__device__ __forceinline__ void riccati_mfma_42(const float* A, const float* B, int mstride, const float* Q2,
                                                const float* R2, const int* hmap, const int* gmap, const float* Hq,
                                                const float* qr, const float* rin, const float* off, float* Kall,
                                                float* kdump, const float* zero4, int N, int nc)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const bool cx = (c & 3) == 0, c2 = c == 2, row0 = g == 0;
    const int j = c >> 2;                       // state of a state column
    const int ua = c == 1 ? 0 : 1;              // input of column 1 or 3
    const bool cu = row0 && (c == 1 || c == 3);
    // lane constants and per-lane LDS pointers (byte strides per step; lanes
    // without a term read the zero block with stride 0)
    const float q2 = cx ? Q2[g * 4 + j] : 0.f;
    const int hm = cx ? hmap[g * 4 + j] : -1;
    const int gm = (!ADJ && c2) ? gmap[g] : -1;
    v4f z1c;
    z1c[0] = q2;
    z1c[1] = cu ? R2[0 * 2 + ua] : 0.f;
    z1c[2] = 0.f;
    z1c[3] = cu ? R2[1 * 2 + ua] : 0.f;
    const char* hp = reinterpret_cast<const char*>(hm >= 0 ? Hq + hm : zero4);
    const unsigned hs = hm >= 0 ? 4u * nc : 0u;
    const char* qp = reinterpret_cast<const char*>(c2 ? qr + g : zero4);
    const unsigned qs = c2 ? 16u : 0u;
    const char* gp = reinterpret_cast<const char*>(gm >= 0 ? Hq + gm : zero4);
    const unsigned gs = gm >= 0 ? 4u * nc : 0u;
    const char* rp = reinterpret_cast<const char*>(c2 && row0 ? rin : zero4);
    const unsigned rs = c2 && row0 ? 8u : 0u;
    const char* fp = reinterpret_cast<const char*>(c2 ? off + g : zero4);
    const unsigned fs = c2 ? 16u : 0u;
    // M_t[4 g][c]: A_t[g][j] at state columns, B_t[g][a] at columns 1 and 3
    const bool mA = cx, mB = c == 1 || c == 3;
    const char* mp = reinterpret_cast<const char*>(mA ? A + g * 4 + j : (mB ? B + g * 2 + ua : zero4));
    const unsigned ms = (mA || mB) ? 4u * mstride : 0u;
    auto at = [](const char* p0, unsigned i, unsigned stride) {
        return reinterpret_cast<const float*>(p0 + __umul24(i, stride));
    };
    const float B2s2 = c2 && row0 ? 1.f : 0.f;
    struct Raw {
        float h, q, gq, f, m;
        float2 r;
    };
    auto fetch = [&](int t, Raw& w) {
        const unsigned tu = t, tp = t >= 1 ? t - 1 : 0;
        w.h = *at(hp, tp, hs);
        w.q = *at(qp, tp, qs);
        w.gq = *at(gp, tp, gs);
        w.f = *at(fp, tu, fs);
        w.m = *at(mp, tu, ms);
        w.r = *reinterpret_cast<const float2*>(at(rp, tu, rs));
    };
    // P^_N: the stage cost of x_N (p in column 2)
    v4f Pm = {0.f, 0.f, 0.f, 0.f};
    Pm[0] = c2 ? *at(qp, N - 1, qs) + *at(gp, N - 1, gs) : q2 + *at(hp, N - 1, hs);
    auto rl = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
    Raw RX, RY;
    fetch(N - 1, RX);
    fetch(N >= 2 ? N - 2 : 0, RY);
    auto step = [&](int t, Raw& R) {
        const float Mc = R.m;
        const float B2s0 = c2 ? R.f : Mc;
        const float Hp = R.h;                         // pose sum of H_t (state entries)
        v4f Z2c = {c2 ? R.q + R.gq : q2, c2 && row0 ? R.r.x : 0.f, 0.f, c2 && row0 ? R.r.y : 0.f};
        if (t == 0) Z2c[0] = c2 ? 0.f : q2;           // h_0 is not used
        v4f zero = {0.f, 0.f, 0.f, 0.f};
        fetch(t >= 2 ? t - 2 : 0, R);
        const v4f W = __builtin_amdgcn_mfma_f32_16x16x4f32(Pm[0], Mc, zero, 0, 0, 0);
        const v4f Z1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mc, W[0], z1c, 0, 0, 0);
        // Quu = Z1 at rows / columns 1 and 3 (lane row 0)
        const float q00 = rl(Z1[1], 1), q01 = rl(Z1[1], 3), q11 = rl(Z1[3], 3);
        v4f Z2 = __builtin_amdgcn_mfma_f32_16x16x4f32(W[0], B2s0, Z2c, 0, 0, 0);
        Z2 = __builtin_amdgcn_mfma_f32_16x16x4f32(W[2], B2s2, Z2, 0, 0, 0);
        const float id = __builtin_amdgcn_rcpf(q00 * q11 - q01 * q01);
        const float i00 = q11 * id, i01 = -q01 * id, i11 = q00 * id;
        // column c of -Quu^{-1} [Qux | qu]
        const float v0 = c2 ? Z2[1] : Z1[1], v1 = c2 ? Z2[3] : Z1[3];
        const float k0 = -(i00 * v0 + i01 * v1), k1 = -(i01 * v0 + i11 * v1);
        {
            // lanes 0, 4, 8, 12 own the gain columns, lane 2 the feedforward
            const bool own = row0 && (cx || c2);
            float* Kt = own ? Kall + t * 10 + (c2 ? 4 : j) : kdump + lane;
            const int ks = own ? 5 : 64;
            Kt[0] = k0;
            Kt[ks] = k1;
        }
        v4f C3;
#pragma unroll
        for (int r = 0; r < 4; ++r) C3[r] = c2 ? Z2[r] : 0.5f * (Z1[r] + Z2[r]);
        C3[0] += Hp;
        C3 = __builtin_amdgcn_mfma_f32_16x16x4f32(Z1[1], row0 ? k0 : 0.f, C3, 0, 0, 0);
        C3 = __builtin_amdgcn_mfma_f32_16x16x4f32(Z1[3], row0 ? k1 : 0.f, C3, 0, 0, 0);
        Pm = C3;
    };
    int t = N - 1;
    for (; t >= 1; t -= 2) {
        step(t, RX);
        step(t - 1, RY);
    }
    if (t == 0) step(0, RX);
}

// Rollout of the 4/2 closed loop x_{t+1} = M_t x_t + c_t, M_t = A + B K_t,
// c_t = B k_t + f_t (gains [K | k] in Kall[t][2][5], offsets f_t in off), by
// a log-depth inclusive scan of the affine maps: G_t <- G_t o G_{t-d} for
// d = 1, 2, 4, ... (Hillis-Steele), one map entry (16 of M, 4 of c) per
// thread, in two buffers of N * 20 floats; then x_{t+1} = G_t(x_0) and
// u_t = K_t x_t + k_t, all steps at once: ceil(log2 N) compositions in
// place of N dependent steps. Writes dX[t][4] =
// x_{t+1} and dU[t][2] = u_t (reverse mode: W[t + 1][4] = x_{t+1}).
template <bool ADJ, int TT>
__device__ __forceinline__ void rollout_scan_42(const float* A, const float* B, int mstride, const float* Kall,
                                                const float* off, const float* x0, float* buf, float* dX, float* dU,
                                                float* W, int N)
{
    const int tid = threadIdx.x;
    const int ne = N * 20;
    float* cur = buf;
    float* nxt = buf + ne;
    for (int e = tid; e < ne; e += TT) {
        const int t = e / 20, q = e % 20;
        const float* K = Kall + t * 10;
        const float* At = A + t * mstride;
        const float* Bt = B + t * mstride;
        float v;
        if (q < 16) {
            const int i = q >> 2, j = q & 3;
            v = At[i * 4 + j] + Bt[i * 2] * K[j] + Bt[i * 2 + 1] * K[5 + j];
        } else {
            const int i = q - 16;
            v = off[t * 4 + i] + Bt[i * 2] * K[4] + Bt[i * 2 + 1] * K[9];
        }
        cur[e] = v;
    }
    __syncthreads();
    for (int d = 1; d < N; d <<= 1) {
        for (int e = tid; e < ne; e += TT) {
            const int t = e / 20, q = e % 20;
            float v = cur[e];
            if (t >= d) {
                // [M_t | c_t] times column j of [G_{t-d} | g_{t-d}] (j = 4: the offset column,
                // plus c_t)
                const float* Mt = cur + t * 20;
                const float* Gp = cur + (t - d) * 20;
                const bool mat = q < 16;
                const int i = mat ? q >> 2 : q - 16;
                const int base = mat ? (q & 3) : 16, stride = mat ? 4 : 1;
                v = mat ? 0.f : Mt[16 + i];
#pragma unroll
                for (int k = 0; k < 4; ++k) v += Mt[i * 4 + k] * Gp[base + k * stride];
            }
            nxt[e] = v;
        }
        __syncthreads();
        float* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    for (int e = tid; e < N * 4; e += TT) {
        const int t = e >> 2, i = e & 3;
        const float* G = cur + t * 20;
        float v = G[16 + i];
#pragma unroll
        for (int k = 0; k < 4; ++k) v += G[i * 4 + k] * x0[k];
        if (ADJ) W[(t + 1) * 4 + i] = v;
        else dX[t * 4 + i] = v;
    }
    if (!ADJ) {
        __syncthreads();
        for (int e = tid; e < N * 2; e += TT) {
            const int t = e >> 1, a = e & 1;
            const float* K = Kall + t * 10 + 5 * a;
            const float* xt = t == 0 ? x0 : dX + (t - 1) * 4;
            float v = K[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v += K[k] * xt[k];
            dU[t * 2 + a] = v;
        }
    }
}

// Riccati sweep for 12 states and 4 inputs in one wave, on 16 x 16 x 4
// FP32 matrix-core tiles (v_mfma_f32_16x16x4f32): no barrier per step. With
// M = [A | B] (12 x 16, zero rows 12-15) and the value function held as the
// 16 x 16 tile P^ (P_{t+1} in rows/columns 0-11, p_{t+1} in column 12), a
// step is
//   W  = P^T M,                                   (4 products)
//   Z1 = blkdiag(H_t, 2Q_u) + M^T W,              (4)
//   Z2 = [H_t | (h_t; r_t)] + W^T [M_x | f^],     (4; f^ = (f_t, 1, 0, 0, 0))
// so that Z1 holds Quu and Qux (rows 12-15), Z2 column 12 holds
// qx = h_t + A^T w and qu = r_t + B^T w with w = P f_t + p (row 12 of W is
// p^T M), and 1/2 (Z1 + Z2) is Qxx exactly symmetric (the two products take
// the same multiplications in the same order, transposed); then the gains
// [K | k] = -Quu^{-1} [Qux | qu] by the 2 x 2 block inverse of Quu (its upper
// triangle, read once per step by every lane; 16 dependent operations where a
// Cholesky factor and two triangular solves take about 40) and
//   P^_t = [Qxx qx] + Qux^T [K | k]               (4, rank 4 in row 3 only).
// Tile layouts of the 16 x 16 x 4 product D = C + A B: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16], and holds D[4 (l / 16) + r][l % 16]
// in register r. Slice s of each product pairs register s of an accumulator
// (k = 4 (l / 16) + s) with the matching entry of M, so a result feeds the
// next product without moving between lanes. The asymmetry that rounding
// leaves in P^ is dropped by the next step's 1/2 (Z1 + Z2).
// Rows 12-15 and columns 13-15 of P^ and W, and columns 13-15 of Z2, carry
// finite values formed anew each step that meet only the zero rows of M
// (and of f^), so they are left unmasked.
// Gains go to Kall[t][4][13] (the other lanes' columns to kdump, 256
// floats); the step terms of step t - 2 (and, TV, the model, from global
// memory) load while step t computes.
template <bool ADJ, bool TV>
__device__ __forceinline__ void riccati_mfma_124(const float* A, const float* B, const float* Ag, const float* Bg,
                                                 int astride, int bstride, int ns, int nu, const float* Q2,
                                                 const float* R2, const int* hmap, const float* Hq, const float* qx,
                                                 const float* rin, const float* off, float* Kall, float* kdump,
                                                 float* mlds, float* qlds, const float* zero4, const float* one4, int N,
                                                 int nc)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const bool c12 = c == 12, r3 = g == 3;
    // lane constants: 2Q_s and 2Q_u entries; per-lane LDS byte addresses and
    // byte strides (per step) of the step terms, lanes without a term
    // reading a block of zeros with stride 0:
    //   H_t - 2Q_s (rows/columns 0-11): the pose sums of step t - 1;
    //   Z2's accumulator: column 12 h_t = qx_{t-1} (rows 0-11, the pose sums
    //     of the gradient already in qx) and r_t (rows 12-15), elsewhere
    //     2Q_s (this lane's slot of qlds);
    //   column 12 of Z2's B operand, f^: f_t (rows 0-11), (1, 0, 0, 0).
    // Z1 starts from blkdiag(2Q_s, 2Q_u) and Z2 from 2Q_s, so that
    // 1/2 (Z1 + Z2) is exactly symmetric with 2Q_s in it.
    v4f z1c;
    const char* hp[4];
    unsigned hs[4];
    float q2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 4 * g + r;
        const bool xx = row < 12 && c < 12;
        const int hm = xx ? hmap[row * 12 + c] : -1;
        q2[r] = xx ? Q2[row * 12 + c] : 0.f;
        z1c[r] = q2[r] + ((row >= 12 && c >= 12) ? R2[(row - 12) * 4 + (c - 12)] : 0.f);
        hp[r] = reinterpret_cast<const char*>(hm >= 0 ? Hq + hm : zero4);
        hs[r] = hm >= 0 ? 4u * nc : 0u;
    }
    *reinterpret_cast<float4*>(qlds + 4 * lane) = make_float4(q2[0], q2[1], q2[2], q2[3]);
    const char* colp = reinterpret_cast<const char*>(c12 ? (r3 ? rin : qx + 4 * g) : qlds + 4 * lane);
    const unsigned col_t = c12 && r3 ? 16u : 0u, col_tp = c12 && !r3 ? 48u : 0u;
    // M_t[4 g + q][c] of this lane: from LDS (one model), or (TV) from
    // A_t = Ag + t astride (n_s x n_s), B_t = Bg + t bstride (n_s x n_u),
    // row-major, loaded from an in-range address (raw; zeroed outside the
    // model by the step that uses it)
    const float* mp[4];
    int mstep[4];
    bool mok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = 4 * g + q, kc = k < ns ? k : ns - 1;
        const bool isA = c < 12;
        const int cu = isA ? 0 : c - 12;
        mp[q] = isA ? Ag + kc * ns + (c < ns ? c : ns - 1) : Bg + kc * nu + (cu < nu ? cu : nu - 1);
        mstep[q] = isA ? astride : bstride;
        mok[q] = k < ns && (isA ? c < ns : cu < nu);
    }
    auto load_m = [&](int t, float (&m)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * g + q;
            if constexpr (TV) m[q] = mp[q][(size_t)t * mstep[q]];
            else m[q] = k < 12 ? (c < 12 ? A[k * 12 + c] : B[k * 4 + (c - 12)]) : 0.f;
        }
    };
    // the B operand of Z2 = [M_x | f^]: one model keeps M in LDS (this
    // lane's slot) so that every lane loads its operand
    if constexpr (!TV) {
        float m0[4];
        load_m(0, m0);
        *reinterpret_cast<float4*>(mlds + 4 * lane) = make_float4(m0[0], m0[1], m0[2], m0[3]);
    }
    const char* b2p = reinterpret_cast<const char*>(c12 ? (r3 ? one4 : off + 4 * g) : (TV ? zero4 : mlds + 4 * lane));
    const unsigned b2s = c12 && !r3 ? 48u : 0u;
    struct Raw {
        float h[4];
        float4 col, b2;
    };
    auto at = [](const char* p, unsigned i, unsigned stride) {
        return reinterpret_cast<const float*>(p + __umul24(i, stride));
    };
    auto fetch = [&](int t, Raw& w) {
        const unsigned tu = t, tp = t >= 1 ? t - 1 : 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) w.h[r] = *at(hp[r], tp, hs[r]);
        w.col = *reinterpret_cast<const float4*>(at(colp, tu, col_t) + __umul24(tp, col_tp) / 4);
        w.b2 = *reinterpret_cast<const float4*>(at(b2p, tu, b2s));
    };
    // P^_N: the stage cost of x_N
    v4f Pm;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 4 * g + r;
        float v = q2[r] + *at(hp[r], N - 1, hs[r]);
        if (c12 && row < 12) v = qx[(N - 1) * 12 + row];
        Pm[r] = v;
    }
    auto rl = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
    // steps alternate between two sets of model registers and step terms,
    // each reloaded two steps ahead of its use
    float MX[4], MY[4];
    Raw RX, RY;
    load_m(N - 1, MX);
    if (TV) load_m(N >= 2 ? N - 2 : 0, MY);
    fetch(N - 1, RX);
    fetch(N >= 2 ? N - 2 : 0, RY);
    auto step = [&](int t, float (&Mraw)[4], Raw& R) {
        // the pose sums of H_t enter only P^_t; H_0 and h_0 are not used
        float Mc[4], B2[4], Hp[4];
        const float b2[4] = {R.b2.x, R.b2.y, R.b2.z, R.b2.w};
        const v4f Z2c = {R.col.x, R.col.y, R.col.z, R.col.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Hp[r] = R.h[r];
            Mc[r] = (!TV || mok[r]) ? Mraw[r] : 0.f;
            B2[r] = (TV && !c12) ? Mc[r] : b2[r];
        }
        v4f W = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) W = __builtin_amdgcn_mfma_f32_16x16x4f32(Pm[q], Mc[q], W, 0, 0, 0);
        v4f Z1 = z1c;
#pragma unroll
        for (int q = 0; q < 4; ++q) Z1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Mc[q], W[q], Z1, 0, 0, 0);
        // Quu^{-1} by 2 x 2 blocks, Quu = [a b; b^T d] (its upper triangle
        // Z1[12 + i][12 + j], lane 60 + j, register i): a^{-1}, E = a^{-1} b
        // and S^{-1} for the Schur complement S = d - b^T E; formed from Z1
        // while the products of Z2 run
        const float a00 = rl(Z1[0], 60), a01 = rl(Z1[0], 61), a11 = rl(Z1[1], 61);
        const float b00 = rl(Z1[0], 62), b01 = rl(Z1[0], 63), b10 = rl(Z1[1], 62), b11 = rl(Z1[1], 63);
        const float d00 = rl(Z1[2], 62), d01 = rl(Z1[2], 63), d11 = rl(Z1[3], 63);
        v4f Z2 = Z2c;
#pragma unroll
        for (int q = 0; q < 4; ++q) Z2 = __builtin_amdgcn_mfma_f32_16x16x4f32(W[q], B2[q], Z2, 0, 0, 0);
        fetch(t >= 2 ? t - 2 : 0, R);
        if constexpr (TV) load_m(t >= 2 ? t - 2 : 0, Mraw);
        const float ia = __builtin_amdgcn_rcpf(a00 * a11 - a01 * a01);
        const float ai00 = a11 * ia, ai01 = -a01 * ia, ai11 = a00 * ia;
        const float e00 = ai00 * b00 + ai01 * b10, e01 = ai00 * b01 + ai01 * b11;
        const float e10 = ai01 * b00 + ai11 * b10, e11 = ai01 * b01 + ai11 * b11;
        const float s00 = d00 - (b00 * e00 + b10 * e10), s01 = d01 - (b00 * e01 + b10 * e11);
        const float s11 = d11 - (b01 * e01 + b11 * e11);
        const float is = __builtin_amdgcn_rcpf(s00 * s11 - s01 * s01);
        const float si00 = s11 * is, si01 = -s01 * is, si11 = s00 * is;
        // column c of -Quu^{-1} [Qux | qu] in row 3 of the wave (Qux column
        // c in Z1, qu in Z2 at c = 12; the other lanes' columns are unused):
        // y = a^{-1} v_1, z = S^{-1} (v_2 - b^T y), x = y - E z
        float v[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) v[a] = c12 ? Z2[a] : Z1[a];
        const float y0 = ai00 * v[0] + ai01 * v[1], y1 = ai01 * v[0] + ai11 * v[1];
        const float rr0 = v[2] - (b00 * y0 + b10 * y1), rr1 = v[3] - (b01 * y0 + b11 * y1);
        const float z0 = si00 * rr0 + si01 * rr1, z1 = si01 * rr0 + si11 * rr1;
        const float x0 = y0 - (e00 * z0 + e01 * z1), x1 = y1 - (e10 * z0 + e11 * z1);
        const float Kh[4] = {-x0, -x1, -z0, -z1};
        {
            // lanes 48-60 own the gain columns; the others write theirs to a
            // slot of their own in kdump
            const bool own = r3 && c <= 12;
            float* Kt = own ? Kall + t * 52 + c : kdump + lane;
            const int ks = own ? 13 : 64;
#pragma unroll
            for (int a = 0; a < 4; ++a) Kt[a * ks] = Kh[a];
        }
        // P^_t (formed at t = 0 too, unused, so that the step has no branch)
        v4f C3;
#pragma unroll
        for (int r = 0; r < 4; ++r) C3[r] = c12 ? Z2[r] : 0.5f * (Z1[r] + Z2[r]) + Hp[r];
#pragma unroll
        for (int q = 0; q < 4; ++q) C3 = __builtin_amdgcn_mfma_f32_16x16x4f32(Z1[q], r3 ? Kh[q] : 0.f, C3, 0, 0, 0);
        Pm = C3;
    };
    int t = N - 1;
    for (; t >= 1; t -= 2) {
        step(t, MX, RX);
        step(t - 1, TV ? MY : MX, RY);
    }
    if (t == 0) step(0, MX, RX);
}

// Trajectory QP of one scenario per workgroup. State/input sizes are padded
// to the compile-time NS >= n_s, NU >= n_u with zero dynamics rows/columns
// and an identity input-cost block, so every small product unrolls.
// TV: the model of step t is read per step (time-varying or per-scenario
// models, or the linearisation of a nonlinear model about the current
// iterate, formed at the start of the kernel).
template <int NS, int NU, bool ADJ, bool TV>
__global__ void __launch_bounds__(traj_threads(NS, NU)) traj_phase_kernel(DevProblem P, int obstacle_free,
                                                                          float* hq_save, TrajAdjoint TA, int cl)
{
    constexpr int TT = traj_threads(NS, NU);
    constexpr int NSU = NS + 1;
    __shared__ float A[NS * NS], B[NS * NU], Q2[NS * NS], R2[NU * NU], cdyn[NS];
    // A^T, B^T (their rows are the columns of A, B), P, (P A)^T, (P B)^T and
    // w: the operands of the sweep's float4 dot products
    __shared__ __align__(16) float AT[NS * NS];
    __shared__ __align__(16) float BT[NU * NS];
    // TV, LDS sweep: A_t^T and B_t^T of the current and the next step (double buffer)
    __shared__ __align__(16) float AT2[TV ? 2 : 1][NS * NS];
    __shared__ __align__(16) float BT2[TV ? 2 : 1][NU * NS];
    __shared__ int hmap[NS * NS], gmap[NS], pmap[NS];
    __shared__ __align__(16) float Pm[NS * NS];
    __shared__ __align__(16) float PAT[NS * NS];
    __shared__ __align__(16) float PBT[NU * NS];
    __shared__ __align__(16) float wv[NS];
    __shared__ float pv[NS];
    __shared__ float Quu[NU * NU], Qux[NU * NS], qu[NU], Qxx[NS * NS], qx[NS];
    __shared__ __align__(16) float xbuf[2][NS];
    __shared__ float x0s[NS];
    __shared__ __align__(16) float zero4[4];   // a float4 of zeros (rollout padding lanes)
    __shared__ __align__(16) float one4[4];    // (1, 0, 0, 0): row 12 of a homogeneous map
    __shared__ float xst[4][16];               // homogeneous start states of the rollout chunks
    extern __shared__ __align__(16) float dyn[];
    const int s = blockIdx.x;
    if (!ADJ && !obstacle_free && P.done[s]) return;
    const int tid = threadIdx.x;
    const int ns = P.n_s, nu = P.n_u, N = P.N, nq = P.nq, nc = P.nc;
    // deviation coordinates about the current iterate (else base point 0)
    const bool dev = !ADJ && !obstacle_free;
    // regions start at 16-byte boundaries (sizes rounded up to 4 floats)
    float* Hq = dyn;                       // [N][nc] reduced contributions
    float* qr = Hq + al4(N * nc);          // [N][NS] stage gradients g_t (reverse: -xbar_t), t = 1..N
    float* Kall = qr + al4(N * NS);        // [N][NU][NS+1] gains [K | k]
    float* sx = Kall;                      // staged before the sweep: [N+1][NS] x (reverse: x^K)
    float* sxr = sx + (N + 1) * NS;        //   [N+1][NS] x_ref
    float* su = sxr + (N + 1) * NS;        //   [N][NU] u (reverse: u^K)
    float* rin = Kall + al4(traj_gain_floats(N, NS, NU));   // [N][NU] input gradients 2 Q_u u^k_t (reverse: -ubar_t)
    float* off = rin + al4(N * NU);        // [N][NS] dynamics offsets f_t (c when the base is 0)
    float* wl = off + al4(N * NS);         // reverse: [N+1][NS] w_t
    float* tvm = wl + (ADJ ? al4((N + 1) * NS) : 0);   // TV, register path: [N][24] padded A_t, B_t
    float4* red4 = reinterpret_cast<float4*>(tvm + (TV && NS == 4 ? al4(N * 24) : 0));   // [TT] chunk sums of split_sums
    // the model of step t in global memory (TV): A_t = Ag + t mts n_s n_s,
    // B_t = Bg + t mts n_s n_u, c_t = cg + t mts n_s (unpadded, row-major);
    // with a nonlinear model (forward pass) the linearisation of this kernel
    const bool sqp = TV && P.model != 0 && dev;
    const float* Ag = P.A_dyn + (size_t)s * P.dyn_ss * ns * ns;
    const float* Bg = P.B_dyn + (size_t)s * P.dyn_ss * ns * nu;
    const float* cg = P.c_dyn + (size_t)s * P.dyn_ss * ns;
    int mts = P.dyn_ts;
    if (sqp) {
        Ag = P.A_lin + (size_t)s * N * ns * ns;
        Bg = P.B_lin + (size_t)s * N * ns * nu;
        mts = 1;
    }
    auto Aat = [&](int t, int i, int j) -> float {
        return (i < ns && j < ns) ? Ag[(size_t)t * mts * ns * ns + i * ns + j] : 0.f;
    };
    auto Bat = [&](int t, int i, int c) -> float {
        return (i < ns && c < nu) ? Bg[(size_t)t * mts * ns * nu + i * nu + c] : 0.f;
    };

    // 0. padded model and cost, pose-coordinate maps; the per-step sums of
    //    the pair contributions (formed beforehand across many workgroups by
    //    sum_partials_kernel, else summed here), their loads overlapping
    //    those of the staged trajectory
    if (tid < 4) {
        zero4[tid] = 0.f;
        one4[tid] = tid == 0 ? 1.f : 0.f;
    }
    if (!ADJ && !obstacle_free && P.hq_pre) {
        for (int e = tid; e < N * nc; e += TT) {
            const float v = P.hq_pre[(size_t)s * N * nc + e];
            Hq[e] = v;
            if (hq_save) hq_save[(size_t)s * N * nc + e] = v;
            if (P.hq_b) P.hq_b[(size_t)s * N * nc + e] = v;
        }
    } else if (!ADJ && !obstacle_free) {
        // the per-step sums over this scenario's workgroup partials (fixed
        // order), four steps per output summed as float4
        const int2 wr0 = P.scen_wg[s];
        const int N4 = (N + 3) / 4;
        split_sums<TT>(
            N4 * nc, wr0.x, wr0.y, (size_t)nc * 16, red4,
            [&](int o) { return reinterpret_cast<const float4*>(P.contrib + (size_t)(o / N4) * 64) + o % N4; },
            [&](int o, float4 v) {
                const int cc = o / N4, t4 = o % N4;
                const float vq[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = 4 * t4 + q;
                    if (t >= N) break;
                    Hq[t * nc + cc] = vq[q];
                    if (hq_save) hq_save[((size_t)s * N + t) * nc + cc] = vq[q];
                    if (P.hq_b) P.hq_b[((size_t)s * N + t) * nc + cc] = vq[q];
                }
            });
    }
    for (int e = tid; e < NS * NS; e += TT) {
        const int i = e / NS, j = e % NS;
        const bool in = i < ns && j < ns;
        A[e] = in ? P.A_dyn[i * ns + j] : 0.f;
        Q2[e] = in ? 2.f * P.Q_s[i * ns + j] : 0.f;
        int ci = -1, cj = -1;
        for (int a = 0; a < nq; ++a) {
            const int qa = a < P.dim ? P.pos_idx[a] : P.att_idx[a - P.dim];
            if (qa == i) ci = a;
            if (qa == j) cj = a;
        }
        int m = -1;
        if (in && ci >= 0 && cj >= 0) {
            const int a = ci < cj ? ci : cj, b2 = ci < cj ? cj : ci;
            m = a * nq - a * (a - 1) / 2 + (b2 - a);     // packed upper-triangle index
        }
        hmap[e] = m;
    }
    for (int e = tid; e < NS * NU; e += TT) {
        const int i = e / NU, j = e % NU;
        const float v = (i < ns && j < nu) ? P.B_dyn[i * nu + j] : 0.f;
        B[e] = v;
        BT[j * NS + i] = v;
    }
    for (int e = tid; e < NS * NS; e += TT) {
        const int i = e / NS, j = e % NS;
        AT[j * NS + i] = (i < ns && j < ns) ? P.A_dyn[i * ns + j] : 0.f;
    }
    for (int e = tid; e < NU * NU; e += TT) {
        const int i = e / NU, j = e % NU;
        R2[e] = (i < nu && j < nu) ? 2.f * P.Q_u[i * nu + j] : (i == j ? 1.f : 0.f);
    }
    // the trajectory the stage terms are formed about, into LDS
    {
        const float* xsrc = ADJ ? TA.xK : (dev ? P.x : nullptr);
        const float* usrc = ADJ ? TA.uK : (dev ? P.u : nullptr);
        const float* xrs = P.x_ref + (size_t)s * (N + 1) * ns;
        for (int e = tid; e < (N + 1) * NS; e += TT) {
            const int t = e / NS, i = e % NS;
            sx[e] = (xsrc && i < ns) ? xsrc[((size_t)s * (N + 1) + t) * ns + i] : 0.f;
            sxr[e] = i < ns ? xrs[t * ns + i] : 0.f;
        }
        for (int e = tid; e < N * NU; e += TT) {
            const int t = e / NU, j = e % NU;
            su[e] = (usrc && j < nu) ? usrc[((size_t)s * N + t) * nu + j] : 0.f;
        }
    }
    if (tid < NS) {
        cdyn[tid] = tid < ns ? P.c_dyn[tid] : 0.f;
        int m = -1, pa = -1;
        for (int a = 0; a < nq; ++a) {
            const int qa = a < P.dim ? P.pos_idx[a] : P.att_idx[a - P.dim];
            if (qa == tid && tid < ns) {
                m = nq * (nq + 1) / 2 + a;
                pa = a;
            }
        }
        gmap[tid] = m;
        pmap[tid] = pa;
    }
    __syncthreads();
    // 1. per-step sums of the pair contributions (fixed order over this
    //    scenario's workgroups) and the stage and input gradients about the
    //    staged trajectory; in reverse mode the stage sums saved by the
    //    forward pass, the state cotangents (pose coordinates summed over this
    //    scenario's workgroups, plus the gradient of the tracking cost at the
    //    last iterate) and the input cotangents
    const int2 wr = P.scen_wg[s];
    if (ADJ) {
        for (int e = tid; e < N * nc; e += TT)
            Hq[e] = TA.hq ? TA.hq[(size_t)s * N * nc + e] : 0.f;
        // four steps per output: the pose partials are summed as float4 (for
        // the pose coordinates; the others have none), plus the gradient of
        // the tracking cost at the last iterate
        const int N4 = (N + 3) / 4;
        auto seed = [&](int t4, int i, float4 part) {
            const float pq[4] = {part.x, part.y, part.z, part.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 4 * t4 + q;
                if (t >= N) break;
                float acc = pq[q];
                if (TA.xK)
#pragma unroll
                    for (int j = 0; j < NS; ++j) acc += Q2[i * NS + j] * (sx[(t + 1) * NS + j] - sxr[(t + 1) * NS + j]);
                qr[t * NS + i] = -acc;
            }
        };
        if (TA.qpart) {
            split_sums<TT>(
                N4 * nq, wr.x, wr.y, (size_t)nq * 16, red4,
                [&](int o) { return reinterpret_cast<const float4*>(TA.qpart + (size_t)(o / N4) * 64) + o % N4; },
                [&](int o, float4 v) {
                    const int a = o / N4;
                    const int i = a < P.dim ? P.pos_idx[a] : P.att_idx[a - P.dim];
                    seed(o % N4, i, v);
                });
        }
        for (int e = tid; e < N4 * NS; e += TT) {
            const int t4 = e / NS, i = e % NS;
            if (!TA.qpart || pmap[i] < 0) seed(t4, i, make_float4(0.f, 0.f, 0.f, 0.f));
        }
        for (int e = tid; e < N * NU; e += TT) {
            const int t = e / NU, j = e % NU;
            float acc = 0.f;
            if (j < nu)
#pragma unroll
                for (int m = 0; m < NU; ++m) acc += R2[j * NU + m] * su[t * NU + m];
            rin[e] = -acc;
        }
        for (int e = tid; e < N * NS; e += TT) off[e] = 0.f;
    } else {
        if (!obstacle_free && P.hq_pre) {
            // read in step 0
        } else if (!obstacle_free) {
            // summed in step 0
        } else {
            for (int e = tid; e < N * nc; e += TT) Hq[e] = 0.f;
        }
        for (int e = tid; e < N * NS; e += TT) {
            const int t = e / NS, i = e % NS;
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < NS; ++j) acc += Q2[i * NS + j] * (sx[(t + 1) * NS + j] - sxr[(t + 1) * NS + j]);
            qr[e] = acc;
        }
        for (int e = tid; e < N * NU; e += TT) {
            const int t = e / NU, j = e % NU;
            float acc = 0.f;
            if (j < nu)
#pragma unroll
                for (int m = 0; m < NU; ++m) acc += R2[j * NU + m] * su[t * NU + m];
            rin[e] = acc;
        }
        // dynamics offsets: the defects of the staged trajectory, in FP64
        // (zero-padded rows and columns contribute nothing)
        if (sqp) {
            // the SQP step: F(x^k_t, u^k_t) and its Jacobian columns, one
            // thread per (step, column); the defect F(x^k_t, u^k_t) - x^k_{t+1}.
            // The sines and cosines of each step are formed once (in the
            // chunk-sum region, free once the sums above are done).
            ModelTrig* mtrig = reinterpret_cast<ModelTrig*>(red4);
            __syncthreads();
            for (int t = tid; t < N; t += TT) model_trig(P.model, sx + t * NS, su + t * NU, mtrig[t]);
            __syncthreads();
            const int nz = ns + nu;
            for (int e = tid; e < N * nz; e += TT) {
                const int t = e / nz, j = e % nz;
                double F[12], col[12];
                // the kernel sizes select the model: 12/4 the quadrotor, 4/2 the bicycle
                constexpr int MODEL = NS == 12 && NU == 4 ? 2 : (NS == 4 && NU == 2 ? 1 : 0);
                model_column<MODEL>(P.model, P.model_par, sx + t * NS, su + t * NU, j, mtrig[t], F, col);
                if (j < ns) {
                    for (int i = 0; i < ns; ++i) P.A_lin[((size_t)s * N + t) * ns * ns + i * ns + j] = (float)col[i];
                } else {
                    for (int i = 0; i < ns; ++i)
                        P.B_lin[((size_t)s * N + t) * ns * nu + i * nu + (j - ns)] = (float)col[i];
                }
                if (j == 0)
                    for (int i = 0; i < NS; ++i)
                        off[t * NS + i] = i < ns ? (float)(F[i] - (double)sx[(t + 1) * NS + i]) : 0.f;
            }
        } else {
            for (int e = tid; e < N * NS; e += TT) {
                const int t = e / NS, i = e % NS;
                double acc = TV ? (i < ns ? (double)cg[(size_t)t * mts * ns + i] : 0.0) : (double)cdyn[i];
                if (dev) {
                    acc -= (double)sx[(t + 1) * NS + i];
#pragma unroll
                    for (int j = 0; j < NS; ++j)
                        acc += (double)(TV ? Aat(t, i, j) : A[i * NS + j]) * (double)sx[t * NS + j];
#pragma unroll
                    for (int j = 0; j < NU; ++j)
                        acc += (double)(TV ? Bat(t, i, j) : B[i * NU + j]) * (double)su[t * NU + j];
                }
                off[e] = (float)acc;
            }
        }
    }
    // the linearisation written above is read back by other threads
    if (sqp) __threadfence_block();
    __syncthreads();
    float* xo = P.x + (size_t)s * (N + 1) * ns;
    float* uo = P.u + (size_t)s * N * nu;
    float* dX = ADJ ? wl : qr;             // forward: dx_t at (t-1) * NS, t = 1..N; reverse: w_t at t * NS
    float* dU = rin;                       // forward: du_t at t * NU
    if constexpr (NS == 4 && NU == 2) {
        // 2. the sweep in the registers of wave 0; 3. the rollout by a scan
        // over all threads, its two buffers in the chunk-sum region
        static_assert(40 * CADMM_MAX_N <= 4 * TT, "rollout scan buffers exceed the chunk-sum region");
        if (tid < 4) {
            float x0d = 0.f;
            if (!ADJ && tid < ns) {
                const float x0v = P.x0[(size_t)s * ns + tid];
                x0d = dev ? x0v - xo[tid] : x0v;
            }
            x0s[tid] = x0d;
            if (ADJ) wl[tid] = 0.f;
        }
        const float* Am = A;
        const float* Bm = B;
        int mstride = 0;
        if constexpr (TV) {
            // padded A_t, B_t of every step into LDS
            for (int e = tid; e < N * 24; e += TT) {
                const int t = e / 24, q = e % 24;
                tvm[e] = q < 16 ? Aat(t, q >> 2, q & 3) : Bat(t, (q - 16) >> 1, (q - 16) & 1);
            }
            __syncthreads();
            Am = tvm;
            Bm = tvm + 16;
            mstride = 24;
        }
        if (tid < 64)
            riccati_mfma_42<ADJ, TV>(Am, Bm, mstride, Q2, R2, hmap, gmap, Hq, qr, rin, off, Kall,
                                     reinterpret_cast<float*>(red4), zero4, N, nc);
        __syncthreads();
        rollout_scan_42<ADJ, TT>(Am, Bm, mstride, Kall, off, x0s, reinterpret_cast<float*>(red4), dX, dU, wl, N);
        __syncthreads();
    } else {
    if constexpr (NS == 12 && NU == 4) {
        // 2. the sweep in wave 0 on matrix-core tiles; the pose sums of the
        //    stage gradients are first added into qr (forward mode), so that
        //    h_t is one load
        if (!ADJ) {
            for (int e = tid; e < N * NS; e += TT) {
                const int m = gmap[e % NS];
                if (m >= 0) qr[e] += Hq[(e / NS) * nc + m];
            }
            __syncthreads();
        }
        if (tid < 64) {
            float* scratch4 = reinterpret_cast<float*>(red4);
            riccati_mfma_124<ADJ, TV>(A, B, Ag, Bg, mts * ns * ns, mts * ns * nu, ns, nu, Q2, R2, hmap, Hq, qr, rin,
                                      off, Kall, scratch4, scratch4 + 256, scratch4 + 512, zero4, one4, N, nc);
        }
        __syncthreads();
    } else {
    // 2. backward Riccati sweep, V_t(x) = 1/2 x^T P x + p^T x, P_N = H_N.
    //    Every phase is one dot product of two contiguous, 16-byte aligned
    //    NS-vectors in LDS per thread (read as float4), so a wave never runs
    //    several output types one after the other:
    //    (a) (P A)^T, (P B)^T (stored transposed, so that (b) reads their
    //        columns as rows), w = P f_t + p;
    //    (b) Quu = 2Q_u + B^T PB, Qux = B^T PA, qu = B^T w + input gradient,
    //        Qxx = H_t + A^T PA, qx = h_t + A^T w (t >= 1), with A^T and B^T
    //        kept in LDS beside A and B;
    //    (c) gains [K | k] = -Quu^{-1} [Qux | qu] and the update
    //        P_t = Qxx + Qux^T K (symmetrised), p_t = qx + Qux^T k: each
    //        thread factors the small Quu itself, so (c) needs no extra barrier.
    // the linear stage terms of the forward pass carry the pose-block
    // gradients of the pair contributions; the adjoint LQ has none
    auto lin = [&](int t, int i) -> float {
        return qr[t * NS + i] + ((!ADJ && gmap[i] >= 0) ? Hq[t * nc + gmap[i]] : 0.f);
    };
    for (int e = tid; e < NS * NS; e += TT) Pm[e] = Q2[e] + (hmap[e] >= 0 ? Hq[(N - 1) * nc + hmap[e]] : 0.f);
    if (tid < NS) pv[tid] = lin(N - 1, tid);
    // phase (a) descriptor of this thread: one output of PA, PB or w
    constexpr int NA = NS * NS + NS * NU + NS;
    int a_type = -1, a_i = 0, a_j = 0;
    if (tid < NS * NS) { a_type = 0; a_i = tid / NS; a_j = tid % NS; }
    else if (tid < NS * NS + NS * NU) { a_type = 1; a_i = (tid - NS * NS) / NU; a_j = (tid - NS * NS) % NU; }
    else if (tid < NA) { a_type = 2; a_i = tid - NS * NS - NS * NU; }
    // phase (b) descriptor: one output of Quu, Qux, qu, Qxx or qx
    constexpr int NB = NU * NU + NU * NS + NU;
    constexpr int NBX = NB + NS * NS + NS;
    int b_type = -1, b_i = 0, b_j = 0;
    if (tid < NU * NU) { b_type = 0; b_i = tid / NU; b_j = tid % NU; }
    else if (tid < NU * NU + NU * NS) { b_type = 1; b_i = (tid - NU * NU) / NS; b_j = (tid - NU * NU) % NS; }
    else if (tid < NB) { b_type = 2; b_i = tid - NU * NU - NU * NS; }
    else if (tid < NB + NS * NS) { b_type = 3; b_i = (tid - NB) / NS; b_j = (tid - NB) % NS; }
    else if (tid < NBX) { b_type = 4; b_i = tid - NB - NS * NS; }
    // phase (c) descriptor: P(i, j) for j >= i, or p(i) (j = NS)
    constexpr int NCP = NS * (NS + 1) / 2 + NS;
    int c_i = -1, c_j = 0;
    if (tid < NCP) {
        int r = tid;
        if (r < NS * (NS + 1) / 2) {
            int i = 0;
            while (r >= NS - i) { r -= NS - i; ++i; }
            c_i = i;
            c_j = i + r;
        } else {
            c_i = r - NS * (NS + 1) / 2;
            c_j = NS;
        }
    }
    // the (b) bias of this thread: its constant part in a register, the
    // step-dependent part read at the top of each step so that its LDS
    // latency hides under phase (a)
    float b_q2 = 0.f;
    int b_hm = -1;
    if (b_type == 0) b_q2 = R2[b_i * NU + b_j];
    else if (b_type == 3) { b_q2 = Q2[b_i * NS + b_j]; b_hm = hmap[b_i * NS + b_j]; }
    else if (b_type == 4) b_hm = ADJ ? -1 : gmap[b_i];
    // TV: thread e < NS NS moves entry (e / NS, e % NS) of A_t into A_t^T,
    // threads NS NS .. NS NS + NS NU - 1 the entries of B_t into B_t^T; the
    // next step's entries are loaded at the top of a step and stored after
    // its phase (c), into the buffer the step after it reads
    const int m_e = tid < NS * NS ? tid : tid - NS * NS;
    const int m_kind = tid < NS * NS ? 0 : (tid < NS * NS + NS * NU ? 1 : -1);
    auto model_entry = [&](int t) -> float {
        return m_kind == 0 ? Aat(t, m_e / NS, m_e % NS) : (m_kind == 1 ? Bat(t, m_e / NU, m_e % NU) : 0.f);
    };
    auto model_store = [&](int buf, float v) {
        if (m_kind == 0) AT2[buf][(m_e % NS) * NS + m_e / NS] = v;
        else if (m_kind == 1) BT2[buf][(m_e % NU) * NS + m_e / NU] = v;
    };
    if constexpr (TV) model_store((N - 1) & 1, model_entry(N - 1));
    __syncthreads();
    for (int t = N - 1; t >= 0; --t) {
        const float* ft = off + t * NS;
        const float* ATc = TV ? AT2[t & 1] : AT;
        const float* BTc = TV ? BT2[t & 1] : BT;
        const float next_m = (TV && t >= 1) ? model_entry(t - 1) : 0.f;
        float bias = b_q2;
        if (b_type == 2) bias = rin[t * NU + b_i];
        else if (b_type == 3 && t >= 1) bias += b_hm >= 0 ? Hq[(t - 1) * nc + b_hm] : 0.f;
        else if (b_type == 4 && t >= 1) bias = qr[(t - 1) * NS + b_i] + (b_hm >= 0 ? Hq[(t - 1) * nc + b_hm] : 0.f);
        // (a)
        if (a_type >= 0) {
            const float* Y = a_type == 0 ? ATc + a_j * NS : (a_type == 1 ? BTc + a_j * NS : ft);
            const float acc = dot_lds<NS>(Pm + a_i * NS, Y, a_type == 2 ? pv[a_i] : 0.f);
            float* O = a_type == 0 ? PAT + a_j * NS + a_i : (a_type == 1 ? PBT + a_j * NS + a_i : wv + a_i);
            *O = acc;
        }
        __syncthreads();
        // (b)
        if (b_type >= 0 && (t >= 1 || b_type <= 2)) {
            // X: column b_i of B (types 0-2) or of A (types 3-4), as a row of B^T / A^T
            const float* X = b_type <= 2 ? BTc + b_i * NS : ATc + b_i * NS;
            const float* Y = b_type == 0 ? PBT + b_j * NS : ((b_type == 1 || b_type == 3) ? PAT + b_j * NS : wv);
            const float acc = dot_lds<NS>(X, Y, bias);
            float* O = b_type == 0 ? Quu + b_i * NU + b_j
                     : b_type == 1 ? Qux + b_i * NS + b_j
                     : b_type == 2 ? qu + b_i
                     : b_type == 3 ? Qxx + b_i * NS + b_j
                                   : qx + b_i;
            *O = acc;
        }
        __syncthreads();
        // (c) gains and, for t >= 1, the value function of step t
        if (c_i >= 0 && (t >= 1 || c_j == c_i || (c_j == NS && c_i == 0))) {
            float L[NU * NU];
#pragma unroll
            for (int q = 0; q < NU * NU; ++q) L[q] = Quu[q];
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                float d = L[j * NU + j];
#pragma unroll
                for (int k2 = 0; k2 < j; ++k2) d -= L[j * NU + k2] * L[j * NU + k2];
                // v_rsq_f32 (about 1 ulp); the diagonal keeps 1 / l_jj
                const float id = __builtin_amdgcn_rsqf(fmaxf(d, 1e-30f));
                L[j * NU + j] = id;
#pragma unroll
                for (int i = j + 1; i < NU; ++i) {
                    float v = L[i * NU + j];
#pragma unroll
                    for (int k2 = 0; k2 < j; ++k2) v -= L[i * NU + k2] * L[j * NU + k2];
                    L[i * NU + j] = v * id;
                }
            }
            // columns c_i and c_j of the gains [K | k] (c_j = NS: feedforward)
            auto gain = [&](int col, float (&r)[NU]) {
#pragma unroll
                for (int i = 0; i < NU; ++i) r[i] = -(col < NS ? Qux[i * NS + col] : qu[i]);
#pragma unroll
                for (int i = 0; i < NU; ++i) {
                    float v = r[i];
#pragma unroll
                    for (int k2 = 0; k2 < i; ++k2) v -= L[i * NU + k2] * r[k2];
                    r[i] = v * L[i * NU + i];
                }
#pragma unroll
                for (int i = NU - 1; i >= 0; --i) {
                    float v = r[i];
#pragma unroll
                    for (int k2 = i + 1; k2 < NU; ++k2) v -= L[k2 * NU + i] * r[k2];
                    r[i] = v * L[i * NU + i];
                }
            };
            float Ki[NU], Kj[NU];
            gain(c_i, Ki);
            gain(c_j, Kj);
            float* Kt = Kall + (size_t)t * NU * NSU;
            // the diagonal threads own the gain columns, thread p(0) the feedforward
            if (c_j == c_i) {
#pragma unroll
                for (int i = 0; i < NU; ++i) Kt[i * NSU + c_i] = Ki[i];
            }
            if (c_j == NS && c_i == 0) {
#pragma unroll
                for (int i = 0; i < NU; ++i) Kt[i * NSU + NS] = Kj[i];
            }
            if (t >= 1) {
                if (c_j < NS) {
                    float aij = Qxx[c_i * NS + c_j] + Qxx[c_j * NS + c_i];
#pragma unroll
                    for (int k2 = 0; k2 < NU; ++k2)
                        aij += Qux[k2 * NS + c_i] * Kj[k2] + Qux[k2 * NS + c_j] * Ki[k2];
                    Pm[c_i * NS + c_j] = 0.5f * aij;
                    Pm[c_j * NS + c_i] = 0.5f * aij;
                } else {
                    float acc = qx[c_i];
#pragma unroll
                    for (int k2 = 0; k2 < NU; ++k2) acc += Qux[k2 * NS + c_i] * Kj[k2];
                    pv[c_i] = acc;
                }
            }
        }
        if (TV && t >= 1) model_store((t - 1) & 1, next_m);
        __syncthreads();
    }
    }
    if (cl && NS == 12) {
    // 3. rollout on the closed loop, dx_{t+1} = (A + B K_t) dx_t + (f_t + B k_t),
    //    in four chunks of the horizon on four waves (one per SIMD):
    //    (a) the maps of all steps as homogeneous tiles G_t = [A + B K_t,
    //        f_t + B k_t; 0 1] (13 x 13 in 16 x 16; rows 0-11 stored, 16
    //        floats each), in parallel;
    //    (b) each wave multiplies out its chunk, Phi = G_{e-1} ... G_s, on
    //        16 x 16 x 4 matrix-core tiles (Phi in the accumulator layout,
    //        which is the B-operand layout of the next product);
    //    (c) the chunk start states x_{s_{w+1}} = Phi_w x_{s_w}, chunk by
    //        chunk (a row sum of the accumulator layout, three barriers);
    //    (d) each wave steps its chunk out from its start state, x in column
    //        0 of the B operand (lane 16 g, register q: entry 4 g + q), the
    //        result landing in the same lanes and registers.
    //    The inputs du_t = K_t dx_t + k_t follow in parallel over t.
    float* Gh = reinterpret_cast<float*>(red4);           // [N][12][16]
    {
        constexpr int NE = 12 * 16, TS = TT / NE;
        const int r = tid % NE, t0 = tid / NE;
        const int i = r / 16, j = r % 16;
        float Bi[NU];
#pragma unroll
        for (int c = 0; c < NU; ++c) Bi[c] = B[i * NU + c];
        const float Aij = j < NS ? A[i * NS + j] : 0.f;
        for (int t = t0; t0 < TS && t < N; t += TS) {
            float acc = 0.f;
            if (j <= NS) {
                const float* Kt = Kall + (size_t)t * NU * NSU + j;
                acc = j < NS ? (TV ? Aat(t, i, j) : Aij) : off[t * NS + i];
#pragma unroll
                for (int c = 0; c < NU; ++c) acc += (TV ? Bat(t, i, c) : Bi[c]) * Kt[c * NSU];
            }
            Gh[((size_t)t * 12 + i) * 16 + j] = acc;
        }
    }
    if (tid < 16) {
        float v = tid == NS ? 1.f : 0.f;
        if (!ADJ && tid < ns) {
            const float x0v = P.x0[(size_t)s * ns + tid];
            v = dev ? x0v - xo[tid] : x0v;
        }
        xst[0][tid] = v;
        if (tid < NS) x0s[tid] = v;
        if (ADJ && tid < NS) wl[tid] = 0.f;
    }
    __syncthreads();
    {
        typedef float v4h __attribute__((ext_vector_type(4)));
        constexpr int NCH = 4;
        const int w = tid >> 6, ci = tid & 15, gi = (tid >> 4) & 3;
        const int cs = (w * N) / NCH, ce = ((w + 1) * N) / NCH;
        // lane (i + 16 g) of the A operand: row i, columns 4 g .. 4 g + 3 of G_t
        const float* gbase = ci < 12 ? Gh + ci * 16 + 4 * gi : ((ci == 12 && gi == 3) ? one4 : zero4);
        const int gstr = ci < 12 ? 12 * 16 : 0;
        auto gload = [&](int t) { return *reinterpret_cast<const float4*>(gbase + (size_t)t * gstr); };
        v4h Phi;
#pragma unroll
        for (int q = 0; q < 4; ++q) Phi[q] = 4 * gi + q == ci ? 1.f : 0.f;
        if (w < NCH && cs < ce) {
            float4 gn = gload(cs);
            for (int t = cs; t < ce; ++t) {
                const float a[4] = {gn.x, gn.y, gn.z, gn.w};
                gn = gload(t + 1 < ce ? t + 1 : t);
                v4h acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], Phi[q], acc, 0, 0, 0);
                Phi = acc;
            }
        }
        for (int c2 = 0; c2 < NCH - 1; ++c2) {
            if (c2 > 0) __syncthreads();
            if (w == c2) {
                // (Phi x)[4 g + q] = sum_j Phi[4 g + q][j] x_j: lane (j + 16 g)
                // holds Phi[4 g + q][j]; sums over the 16 lanes of a row
                const float xj = xst[c2][ci];
                float p[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float v = Phi[q] * xj;
                    v += row_ror<8>(v);
                    v += row_ror<4>(v);
                    v += row_ror<2>(v);
                    v += row_ror<1>(v);
                    p[q] = v;
                }
                if (ci == 0) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) xst[c2 + 1][4 * gi + q] = p[q];
                }
            }
        }
        __syncthreads();
        if (w < NCH && cs < ce) {
            float xb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) xb[q] = ci == 0 ? xst[w][4 * gi + q] : 0.f;
            float4 gn = gload(cs);
            for (int t = cs; t < ce; ++t) {
                const float a[4] = {gn.x, gn.y, gn.z, gn.w};
                gn = gload(t + 1 < ce ? t + 1 : t);
                v4h acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], xb[q], acc, 0, 0, 0);
                if (ci == 0 && gi < 3) {
                    float* o = ADJ ? wl + (t + 1) * NS + 4 * gi : dX + t * NS + 4 * gi;
                    *reinterpret_cast<float4*>(o) = make_float4(acc[0], acc[1], acc[2], acc[3]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) xb[q] = acc[q];
            }
        }
    }
    __syncthreads();
    if (!ADJ) {
        for (int e = tid; e < N * NU; e += TT) {
            const int t = e / NU, c = e % NU;
            const float* Kt = Kall + (size_t)t * NU * NSU + c * NSU;
            const float* xt = t == 0 ? x0s : dX + (t - 1) * NS;
            float u = Kt[NS];
#pragma unroll
            for (int k2 = 0; k2 < NS; ++k2) u += Kt[k2] * xt[k2];
            dU[e] = u;
        }
        __syncthreads();
    }
    } else if (cl) {
    // 3. rollout on the closed loop, dx_{t+1} = (A + B K_t) dx_t + (f_t + B k_t):
    //    the matrices of all steps are formed first, in parallel, so that a
    //    step is one float4 dot product per state (thread i owns dx_i); the
    //    inputs du_t = K_t dx_t + k_t follow in parallel over t.
    float* Acl = reinterpret_cast<float*>(red4);          // [N][NS][NS]
    float* Ccl = Acl + (size_t)N * NS * NS;               // [N][NS]
    {
        // thread -> entry (i, j) of every step t = t0, t0 + TS, ... (j = NS:
        // the offset), the one-model rows of A and B in registers
        constexpr int NE = NS * (NS + 1), TS = TT / NE;
        const int r = tid % NE, t0 = tid / NE;
        const int i = r / (NS + 1), j = r % (NS + 1);
        float Bi[NU];
#pragma unroll
        for (int c = 0; c < NU; ++c) Bi[c] = B[i * NU + c];
        const float Aij = j < NS ? A[i * NS + j] : 0.f;
        for (int t = t0; t0 < TS && t < N; t += TS) {
            const float* Kt = Kall + (size_t)t * NU * NSU + j;
            float acc = j < NS ? (TV ? Aat(t, i, j) : Aij) : off[t * NS + i];
#pragma unroll
            for (int c = 0; c < NU; ++c) acc += (TV ? Bat(t, i, c) : Bi[c]) * Kt[c * NSU];
            if (j < NS) Acl[((size_t)t * NS + i) * NS + j] = acc;
            else Ccl[t * NS + i] = acc;
        }
    }
    if (tid < NS) {
        float v = 0.f;
        if (!ADJ && tid < ns) {
            const float x0v = P.x0[(size_t)s * ns + tid];
            v = dev ? x0v - xo[tid] : x0v;
        }
        xbuf[0][tid] = v;
        x0s[tid] = v;
        if (ADJ) wl[tid] = 0.f;
    }
    __syncthreads();
    // the steps in wave 0 on 16 x 16 x 4 matrix-core tiles, without
    // barriers: dx_t is column 0 of the B operand (lane 16 g, register s:
    // entry 4 g + s), so that D = [c_t | 0] + A^cl_t [dx_t | 0] leaves
    // dx_{t+1} in the same lanes and registers; slice s takes column
    // 4 g + s of A^cl_t (lane i + 16 g, one float4 of row i). The rows of
    // step t + 1 load while step t computes.
    if (tid < 64) {
        typedef float v4r __attribute__((ext_vector_type(4)));
        const int ci = tid & 15, gi = tid >> 4;
        const bool arow = ci < NS && 4 * gi < NS;
        const bool xl = ci == 0 && 4 * gi < NS;
        // lanes outside the tile read the zero block (stride 0)
        const float* abase = arow ? Acl + ci * NS + 4 * gi : zero4;
        const float* cbase = xl ? Ccl + 4 * gi : zero4;
        const int astr = arow ? NS * NS : 0, cstr = xl ? NS : 0;
        struct Row {
            float4 a, c;
        };
        auto load = [&](int t, Row& r) {
            const int tc = t < N ? t : N - 1;
            r.a = *reinterpret_cast<const float4*>(abase + (size_t)tc * astr);
            r.c = *reinterpret_cast<const float4*>(cbase + tc * cstr);
        };
        float xb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xb[q] = xl ? xbuf[0][4 * gi + q] : 0.f;
        Row RA, RB;
        load(0, RA);
        load(1, RB);
        auto step = [&](int t, Row& R) {
            const float a[4] = {R.a.x, R.a.y, R.a.z, R.a.w};
            v4r acc = {R.c.x, R.c.y, R.c.z, R.c.w};
            load(t + 2, R);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], xb[q], acc, 0, 0, 0);
            // lanes 0, 16, 32 (and 48 when NS = 16) own dx_{t+1}
            float* o = ADJ ? wl + (t + 1) * NS + 4 * gi : dX + t * NS + 4 * gi;
            if (xl) *reinterpret_cast<float4*>(o) = make_float4(acc[0], acc[1], acc[2], acc[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) xb[q] = acc[q];
        };
        int t = 0;
        for (; t + 1 < N; t += 2) {
            step(t, RA);
            step(t + 1, RB);
        }
        if (t < N) step(t, RA);
    }
    __syncthreads();
    if (!ADJ) {
        for (int e = tid; e < N * NU; e += TT) {
            const int t = e / NU, c = e % NU;
            const float* Kt = Kall + (size_t)t * NU * NSU + c * NSU;
            const float* xt = t == 0 ? x0s : dX + (t - 1) * NS;
            float u = Kt[NS];
#pragma unroll
            for (int k2 = 0; k2 < NS; ++k2) u += Kt[k2] * xt[k2];
            dU[e] = u;
        }
        __syncthreads();
    }
    } else {
    // 3. rollout dx_{t+1} = A dx + B (K dx + k) + f_t; thread i owns dx_i
    //    (rows of A and B in registers), threads NS..NS+NU-1 the inputs. The
    //    deviations stay in LDS (forward: over qr and rin, dead after the
    //    sweep; reverse: w in wl) and are written out by one parallel pass.
    float Ar[NS], Br[NU];
    const int row = tid < NS ? tid : 0;
#pragma unroll
    for (int k2 = 0; k2 < NS; ++k2) Ar[k2] = A[row * NS + k2];
#pragma unroll
    for (int j = 0; j < NU; ++j) Br[j] = B[row * NU + j];
    if (tid < NS) {
        float v = 0.f;
        if (!ADJ && tid < ns) {
            const float x0v = P.x0[(size_t)s * ns + tid];
            v = dev ? x0v - xo[tid] : x0v;
        }
        xbuf[0][tid] = v;
        if (ADJ) wl[tid] = 0.f;
    }
    __syncthreads();
    for (int t = 0; t < N; ++t) {
        const float* xc = xbuf[t & 1];
        const float* Kt = Kall + (size_t)t * NU * NSU;
        if (TV && tid < NS) {
#pragma unroll
            for (int k2 = 0; k2 < NS; ++k2) Ar[k2] = Aat(t, row, k2);
#pragma unroll
            for (int j = 0; j < NU; ++j) Br[j] = Bat(t, row, j);
        }
        if (tid < NS + NU) {
            float xr[NS];
#pragma unroll
            for (int k2 = 0; k2 < NS; ++k2) xr[k2] = xc[k2];
            float uu[NU];
#pragma unroll
            for (int j = 0; j < NU; ++j) {
                float v = Kt[j * NSU + NS];
#pragma unroll
                for (int k2 = 0; k2 < NS; ++k2) v += Kt[j * NSU + k2] * xr[k2];
                uu[j] = v;
            }
            if (tid < NS) {
                float acc = off[t * NS + tid];
#pragma unroll
                for (int k2 = 0; k2 < NS; ++k2) acc += Ar[k2] * xr[k2];
#pragma unroll
                for (int j = 0; j < NU; ++j) acc += Br[j] * uu[j];
                xbuf[(t + 1) & 1][tid] = acc;
                if (ADJ) wl[(t + 1) * NS + tid] = acc;
                else dX[t * NS + tid] = acc;
            } else if (!ADJ) {
                const int j = tid - NS;
                float v = 0.f;
#pragma unroll
                for (int q = 0; q < NU; ++q) v = q == j ? uu[q] : v;
                dU[t * NU + j] = v;
            }
        }
        __syncthreads();
    }
    }
    }
    if (!ADJ) {
        // x_t = x^k_t + dx_t (t = 1..N), u_t = u^k_t + du_t, x_0 = x0
        for (int e = tid; e < N * ns; e += TT) {
            const int t = e / ns, i = e % ns;
            float* xp = xo + (t + 1) * ns + i;
            *xp = (dev ? *xp : 0.f) + dX[t * NS + i];
        }
        for (int e = tid; e < N * nu; e += TT) {
            const int t = e / nu, j = e % nu;
            float* up = uo + t * nu + j;
            *up = (dev ? *up : 0.f) + dU[t * NU + j];
        }
        if (tid < ns) xo[tid] = P.x0[(size_t)s * ns + tid];
        return;
    }
    // 4. reverse mode: w_t out, zbar_t = xbar_t - H_t w_t (stored over qr),
    //    then x0bar = sum_t (A^T)^t zbar_t by a Horner sweep from t = N down
    //    to 1 (one barrier per step, double-buffered)
    for (int e = tid; e < N * ns; e += TT) {
        const int t = e / ns, i = e % ns;
        TA.w[((size_t)s * N + t) * ns + i] = wl[(t + 1) * NS + i];
    }
    for (int e = tid; e < N * NS; e += TT) {
        const int t = e / NS, i = e % NS;
        const float* wt = wl + (t + 1) * NS;
        float acc = -qr[e];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int m = hmap[i * NS + j];
            acc -= (Q2[i * NS + j] + (m >= 0 ? Hq[t * nc + m] : 0.f)) * wt[j];
        }
        qr[e] = acc;
    }
    if (tid < NS) xbuf[0][tid] = 0.f;
    __syncthreads();
    int cur = 0;
    for (int t = N - 1; t >= 0; --t) {
        if (tid < NS) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < NS; ++j)
                acc += (TV ? Aat(t, j, tid) : A[j * NS + tid]) * (xbuf[cur][j] + qr[t * NS + j]);
            xbuf[cur ^ 1][tid] = acc;
        }
        cur ^= 1;
        __syncthreads();
    }
    if (tid < ns) TA.gx0[(size_t)s * ns + tid] += (double)xbuf[cur][tid];
}

// Per-step sums of the pair contributions of scenarios with many pair-phase
// workgroups, spread over many workgroups instead of the one of the
// trajectory kernel (which then reads the sums): workgroup (s, c) sums
// coordinate c of every step over the scenario's workgroup partials, wave q
// the workgroups w = first + q (mod 16) in order, the 16 wave partials then
// in order (a fixed order: runs are bitwise repeatable).
constexpr int kSumWaves = 16;
__global__ void __launch_bounds__(64 * kSumWaves) sum_partials_kernel(DevProblem P, float* out)
{
    __shared__ float red[kSumWaves][64];
    const int s = blockIdx.x / P.nc, c = blockIdx.x % P.nc;
    const int q = threadIdx.x / 64, t = threadIdx.x % 64;
    const int2 wr = P.scen_wg[s];
    float acc = 0.f;
    if (!P.done[s] && t < P.N) {
        // eight loads in flight ahead of their adds (same order of the adds)
        const float* src = P.contrib + (size_t)c * 64 + t;
        const size_t ws = (size_t)P.nc * 64;
        int w = wr.x + q;
        for (; w + 7 * kSumWaves < wr.y; w += 8 * kSumWaves) {
            float a[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = src[(size_t)(w + k * kSumWaves) * ws];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc += a[k];
        }
        for (; w < wr.y; w += kSumWaves) acc += src[(size_t)w * ws];
    }
    red[q][t] = acc;
    __syncthreads();
    if (q == 0 && t < P.N && !P.done[s]) {
        float v = red[0][t];
        for (int k = 1; k < kSumWaves; ++k) v += red[k][t];
        out[((size_t)s * P.N + t) * P.nc + c] = v;
    }
}

template <bool ADJ, bool TV>
static hipError_t launch_traj_tv(const DevProblem& P, int obstacle_free, float* hq_save, const TrajAdjoint& TA,
                                 hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    dim3 g(P.n_scen);
    // closed-loop rollout where its matrices fit in the 64 KB of LDS beside
    // the rest (the static arrays take 5.3 KB at 12/4, 10.1 KB at 16/8)
    auto cl_fits = [&](int NS, int NU) {
        const size_t budget = NS <= 12 ? 56 * 1024 : 52 * 1024;
        return (size_t)traj_dyn_floats(P.N, NS, NU, P.nc, ADJ, true) * sizeof(float) <= budget;
    };
    if (P.n_s <= 4 && P.n_u <= 2) {
        const dim3 b(traj_threads(4, 2));
        CADMM_LAUNCH((traj_phase_kernel<4, 2, ADJ, TV>), g, b,
                     sizeof(float) * traj_dyn_floats(P.N, 4, 2, P.nc, ADJ, false, TV), st, e0, e1, P, obstacle_free,
                     hq_save, TA, 0);
    } else if (P.n_s <= 12 && P.n_u <= 4) {
        const dim3 b(traj_threads(12, 4));
        const bool cl = cl_fits(12, 4);
        CADMM_LAUNCH((traj_phase_kernel<12, 4, ADJ, TV>), g, b,
                     sizeof(float) * traj_dyn_floats(P.N, 12, 4, P.nc, ADJ, cl, TV), st, e0, e1, P, obstacle_free,
                     hq_save, TA, cl ? 1 : 0);
    } else {
        const dim3 b(traj_threads(16, 8));
        const bool cl = cl_fits(16, 8);
        CADMM_LAUNCH((traj_phase_kernel<16, 8, ADJ, TV>), g, b,
                     sizeof(float) * traj_dyn_floats(P.N, 16, 8, P.nc, ADJ, cl, TV), st, e0, e1, P, obstacle_free,
                     hq_save, TA, cl ? 1 : 0);
    }
    return hipGetLastError();
}

// Per-step models (time-varying, per scenario, or a nonlinear model) take
// the TV instantiation; one time-invariant model keeps its matrices in LDS
// and registers for the whole sweep.
template <bool ADJ>
static hipError_t launch_traj(const DevProblem& P, int obstacle_free, float* hq_save, const TrajAdjoint& TA,
                              hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    if (P.dyn_ts != 0 || P.dyn_ss != 0 || P.model != 0)
        return launch_traj_tv<ADJ, true>(P, obstacle_free, hq_save, TA, st, e0, e1);
    return launch_traj_tv<ADJ, false>(P, obstacle_free, hq_save, TA, st, e0, e1);
}

hipError_t launch_traj_phase(const DevProblem& P, int obstacle_free, hipStream_t st, float* hq_save, hipEvent_t e0,
                             hipEvent_t e1)
{
    // up to three kernels (the per-step sums spread over many workgroups, the
    // sweep, the bounded QP); the events bracket all of them
    const bool pre = P.hq_pre && !obstacle_free;
    if (pre) {
        const dim3 g(P.n_scen * P.nc), b(64 * kSumWaves);
        CADMM_LAUNCH(sum_partials_kernel, g, b, 0, st, e0, nullptr, P, const_cast<float*>(P.hq_pre));
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipEvent_t t0 = pre ? nullptr : e0;
    if (!P.has_bounds) return launch_traj<false>(P, obstacle_free, hq_save, TrajAdjoint{}, st, t0, e1);
    const hipError_t err = launch_traj<false>(P, obstacle_free, hq_save, TrajAdjoint{}, st, t0, nullptr);
    if (err != hipSuccess) return err;
    return launch_traj_bounds(P, obstacle_free, st, e1);
}

hipError_t launch_traj_adjoint(const DevProblem& P, const TrajAdjoint& TA, hipStream_t st)
{
    return launch_traj<true>(P, 0, nullptr, TA, st);
}

} // namespace cadmm
