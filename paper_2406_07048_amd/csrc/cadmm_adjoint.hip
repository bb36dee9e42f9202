// gfx950 reverse-pass kernels of the ADMM collision-avoidance path (arXiv
// 2406.07048): the cotangent of the tracking cost after K unrolled
// iterations (Sec. IV-B: pair QPs, trajectory QP, multiplier update) with
// respect to the obstacle offsets d and the initial states x_0.
//
// One step k -> k+1 of the iteration is reversed by two launches:
//   - the trajectory kernel in reverse mode (one adjoint LQ per scenario,
//     giving w, see cadmm_traj.hip), then
//   - the reverse pair kernel below, one wavefront per pair block, lane t-1
//     = pair t, which for every pair at the pose of x^k
//       (a) reverses the pair's stage terms H_t += sigma J^T J,
//           h_t += sigma J^T (e - J q^k) of the trajectory QP,
//       (b) reverses the proximal pair QP on its free set by implicit
//           differentiation of its (dim+2)-dimensional dual optimality
//           system, and
//       (c) reverses the multiplier update zeta^k = zeta^{k-1} + T(x^k, y^k),
//           xi^k = xi^{k-1} + R(x^k, y^k) of the previous step, whose pose
//           is the same x^k.
// Pose cotangents are summed over the waves of a workgroup in LDS (fixed
// order) and per workgroup into a partial buffer that the next reverse
// trajectory launch sums per step; offset cotangents are summed over the
// lanes of a wave and accumulated in FP64 per (part, face), a slot owned by
// exactly one pair block. No float atomics: the pass is bitwise repeatable.
#include "cadmm.h"
#include "cadmm_device.h"

namespace cadmm {

// ------------------------------------------------------------------------
// second derivatives of R(s) for the ZYX Euler attitude: R = Rz(psi)
// Ry(theta) Rx(phi), and the k-th derivative of a one-axis factor has the
// entries cos(a + k pi/2), sin(a + k pi/2) in its rotating block and the
// axis entry 1 for k = 0, 0 otherwise.
// ------------------------------------------------------------------------

struct AxisD {
    float c, s, one;
};

__device__ __forceinline__ AxisD axis_deriv(float c, float s, int k)
{
    AxisD r;
    r.c = k == 0 ? c : (k == 1 ? -s : -c);
    r.s = k == 0 ? s : (k == 1 ? c : -s);
    r.one = k == 0 ? 1.f : 0.f;
    return r;
}

// u^T (d2 R / d att_a d att_b) v for the attitude coordinates a, b in
// (phi, theta, psi) order; cs holds (cos, sin) of phi, theta, psi.
__device__ __forceinline__ float euler_dd_form(const float (&cs)[6], int a, int b, const float* u, const float* v)
{
    const AxisD X = axis_deriv(cs[0], cs[1], (a == 0) + (b == 0));
    const AxisD Y = axis_deriv(cs[2], cs[3], (a == 1) + (b == 1));
    const AxisD Z = axis_deriv(cs[4], cs[5], (a == 2) + (b == 2));
    // p = Rx' v
    const float p0 = X.one * v[0], p1 = X.c * v[1] - X.s * v[2], p2 = X.s * v[1] + X.c * v[2];
    // q = Ry' p
    const float q0 = Y.c * p0 + Y.s * p2, q1 = Y.one * p1, q2 = -Y.s * p0 + Y.c * p2;
    // Rz'^T u
    const float r0 = Z.c * u[0] + Z.s * u[1], r1 = -Z.s * u[0] + Z.c * u[1], r2 = Z.one * u[2];
    return r0 * q0 + r1 * q1 + r2 * q2;
}

// Jacobian of (T, R) of one pair in the pose coordinates (position,
// attitude) from cbar = sum_l mu_l c_l (world frame): T depends on the
// position through d' = d - C pos and R on the attitude through R^T cbar.
template <int DIM>
__device__ __forceinline__ void pair_jacobian(const Pose<DIM>& ps, const float (&cb)[DIM], const float* o,
                                              float (&J)[(DIM + 1) * Pose<DIM>::NQ])
{
    constexpr int NQ = Pose<DIM>::NQ, NATT = Pose<DIM>::NATT;
#pragma unroll
    for (int i = 0; i < (DIM + 1) * NQ; ++i) J[i] = 0.f;
#pragma unroll
    for (int c = 0; c < DIM; ++c) J[c] = -cb[c];
#pragma unroll
    for (int a = 0; a < NATT; ++a) {
        const float* dRa = ps.dR + a * DIM * DIM;
        float acc = 0.f;
#pragma unroll
        for (int r = 0; r < DIM; ++r)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc += cb[r] * dRa[r * DIM + c] * o[c];
        J[DIM + a] = -acc;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            float v = 0.f;
#pragma unroll
            for (int r = 0; r < DIM; ++r) v += dRa[r * DIM + c] * cb[r];
            J[(1 + c) * NQ + DIM + a] = v;
        }
    }
}

template <int DIM>
__device__ __forceinline__ float dot3(const float4& f, const float* v)
{
    return f.x * v[0] + f.y * v[1] + (DIM == 3 ? f.z * v[DIM - 1] : 0.f);
}

// ------------------------------------------------------------------------
// reverse pair kernel (see the file comment). Per lane, with rows
//   lambda_k: w_k = (0, a_k, -b_k),  mu_l: w_l = (d'_l, R^T c_l, 0),
//   gamma:    w = (1, 0, 0),          s_l = 1 / (eps D_l), D_l = ||K_l||^2,
// the pair QP's solution on its free set F = {l : y_l > 0} is
//   y_l = yhat_l - s_l w_l.z,   H z = sum_F yhat_l w_l + (bhat, 1),
//   H = diag(1, .., 1, 0) + sum_F s_l w_l w_l^T,
// so for the cotangent ybar: abar = H^{-1} (-sum_F ybar_l s_l w_l),
//   g_l = ybar_l + w_l.abar = cotangent of yhat_l, bhat_bar = abar[0..dim],
//   wbar_l = y_l abar - s_l g_l z, sbar_l = -(w_l.z) g_l,
// and D_l, d'_l, R carry these back to the offsets and the pose.
// ------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(512) pair_adjoint_kernel(DevProblem P, PairAdjoint A)
{
    constexpr int NV = DIM + 2;
    constexpr int D1 = DIM + 1;
    constexpr int NATT = Pose<DIM>::NATT;
    constexpr int NQ = Pose<DIM>::NQ;
    constexpr int MF = CADMM_MAX_PART_FACES + CADMM_MAX_OBS_FACES;
    extern __shared__ __align__(16) float lds[];
    const int W = blockDim.x >> 6;
    // per wave: the block's faces [MF] float4 and obstacle offsets in FP64
    // [CADMM_MAX_OBS_FACES], then the pose partials [W][NQ][64]
    float4* faces_all = reinterpret_cast<float4*>(lds);
    double* d64_all = reinterpret_cast<double*>(faces_all + W * MF);
    float* red = reinterpret_cast<float*>(d64_all + W * CADMM_MAX_OBS_FACES);
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int N = P.N;
    const float eps = P.eps_prox, sg = P.sigma;
    const int t = lane + 1;
    const bool act = t <= N;
    const int tc = act ? t : N;             // lanes past the horizon mirror the last pair, writes masked

    for (int wg = blockIdx.x; wg < P.n_wg; wg += gridDim.x) {
        const int4 item = P.wg_items[wg];
        const int s = uniform(item.x);
        const int b = uniform(item.y + wave);
        float qbar[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a) qbar[a] = 0.f;
        // the block's faces and FP64 offsets into this wave's LDS slot (read
        // by all three row passes)
        float4* fl = faces_all + wave * MF;
        double* dl = d64_all + wave * CADMM_MAX_OBS_FACES;
        if (b < item.z) {
            const int4 bk = P.blocks[b];
            const int f0 = P.part_face_ptr[bk.y], nf = P.part_face_ptr[bk.y + 1] - f0;
            const int g0 = P.obs_face_ptr[bk.z], ng = P.obs_face_ptr[bk.z + 1] - g0;
            if (lane < nf) fl[lane] = P.part_faces[f0 + lane];
            if (lane < ng) {
                fl[CADMM_MAX_PART_FACES + lane] = P.obs_faces[g0 + lane];
                dl[lane] = P.obs_d64[g0 + lane];
            }
        }
        __syncthreads();
        if (b < item.z) {
            const int4 blk = P.blocks[b];
            const int part = uniform(blk.y), obs = uniform(blk.z);
            const int fr0 = uniform(P.part_face_ptr[part]);
            const int nr = uniform(P.part_face_ptr[part + 1] - fr0);
            const int fo0 = uniform(P.obs_face_ptr[obs]);
            const int no = uniform(P.obs_face_ptr[obs + 1] - fo0);
            const float4* cl = P.obs_dc + fo0;   // rounding of the obstacle's FP32 normals
            const int yoff = uniform(P.block_yoff[b]);
            const float4* rf = fl;
            const float4* of = fl + CADMM_MAX_PART_FACES;
            const size_t col = (size_t)yoff + (tc - 1);
            const float* yn = A.yn + col;
            const float* yk = A.yk + col;
            float* yb = A.yb + col;
            Pose<DIM> ps;
            make_pose<DIM>(P, A.xk + ((size_t)s * (N + 1) + tc) * P.n_s, part, ps);
            const float* o = P.part_off + part * 3;
            float xq[NQ], wq[NQ];
            {
                const float* xn = A.xn + ((size_t)s * (N + 1) + tc) * P.n_s;
                const float* wt = A.w + ((size_t)s * N + tc - 1) * P.n_s;
#pragma unroll
                for (int a = 0; a < NQ; ++a) {
                    const int idx = a < DIM ? P.pos_idx[a] : P.att_idx[a - DIM];
                    xq[a] = xn[idx];
                    wq[a] = wt[idx];
                }
            }
            const size_t pr = (size_t)b * N + tc - 1;
            const float zeta = A.zk[pr];
            float xi[DIM], xib_in[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                xi[r] = A.xik[((size_t)b * DIM + r) * N + tc - 1];
                xib_in[r] = A.xib[((size_t)b * DIM + r) * N + tc - 1];
            }
            const float zb_in = A.zb[pr];

            // ---- (a) stage terms at (x^k, y^{k+1}) ----
            float Al[DIM] = {}, Sd = 0.f, cb[DIM] = {};
            for (int k = 0; k < nr; ++k) {
                const float4 f = rf[k];
                const float y = yn[(size_t)k * N];
                Al[0] += y * f.x;
                Al[1] += y * f.y;
                if (DIM == 3) Al[DIM - 1] += y * f.z;
            }
            for (int l = 0; l < no; ++l) {
                const float4 f = of[l];
                const float y = yn[(size_t)(nr + l) * N];
                Sd += face_offset(dl, l, f, cl[l], ps.pos64, ps.pos, DIM) * y;
                cb[0] += y * f.x;
                cb[1] += y * f.y;
                if (DIM == 3) cb[DIM - 1] += y * f.z;
            }
            const float yg1 = yn[(size_t)(nr + no) * N];
            float J[D1 * NQ];
            pair_jacobian<DIM>(ps, cb, o, J);
            // residual r = (T + zeta, R + xi) at (x^k, y^{k+1})
            float e[D1];
            e[0] = 1.f + Sd + yg1 + zeta;
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = Al[r] + xi[r];
#pragma unroll
                for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * cb[m];
                e[1 + r] = acc;
            }
            // cotangents of the stage terms: Hbar = -(w x^T + x w^T)/2 and
            // hbar = -w at x = x^{k+1}, through H += sigma J^T J and
            // h += sigma J^T (r - J q^k):
            //   Jbar = sigma (J (Hbar + Hbar^T) + (r - J q^k) hbar^T - (J hbar) q^kT)
            //        = sigma ((J hbar) dq^T - (r + J dq) w^T),  dq = x^{k+1} - x^k
            // (pose coordinates), the form without cancellation
            float Jh[D1], Jdq[D1], dq[NQ];
#pragma unroll
            for (int a = 0; a < NQ; ++a) dq[a] = xq[a] - ps.q[a];
#pragma unroll
            for (int m = 0; m < D1; ++m) {
                float a1 = 0.f, a2 = 0.f;
#pragma unroll
                for (int a = 0; a < NQ; ++a) {
                    a1 -= J[m * NQ + a] * wq[a];
                    a2 += J[m * NQ + a] * dq[a];
                }
                Jh[m] = a1;
                Jdq[m] = a2;
            }
            float Jb[D1 * NQ];
#pragma unroll
            for (int m = 0; m < D1; ++m)
#pragma unroll
                for (int a = 0; a < NQ; ++a) Jb[m * NQ + a] = sg * (Jh[m] * dq[a] - (e[m] + Jdq[m]) * wq[a]);
            // rbar = sigma J hbar: cotangent of (T + zeta, R + xi). Its pose
            // term J^T rbar cancels the -sigma J^T J hbar that the -J q^k of
            // the linear stage term contributes, so neither is formed.
            float rbar[D1];
#pragma unroll
            for (int m = 0; m < D1; ++m) rbar[m] = sg * Jh[m];
            // through J: cbar (world) and the attitude (second derivatives)
            float cbb[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) cbb[c] = -Jb[c];
#pragma unroll
            for (int a = 0; a < NATT; ++a) {
                const float* dRa = ps.dR + a * DIM * DIM;
                const float j0 = Jb[DIM + a];
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) acc += dRa[r * DIM + c] * (Jb[(1 + c) * NQ + DIM + a] - j0 * o[c]);
                    cbb[r] += acc;
                }
            }
            if constexpr (DIM == 2) {
                // d2R/dtheta2 = -R
                float acc = 0.f;
#pragma unroll
                for (int r = 0; r < 2; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) acc -= cb[r] * ps.R[r * 2 + c] * (Jb[(1 + c) * NQ + 2] - Jb[2] * o[c]);
                qbar[2] += acc;
            } else {
                float cs[6];
                sincosf(ps.q[3], &cs[1], &cs[0]);
                sincosf(ps.q[4], &cs[3], &cs[2]);
                sincosf(ps.q[5], &cs[5], &cs[4]);
#pragma unroll
                for (int bq = 0; bq < 3; ++bq) {
                    float acc = 0.f;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        float va[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) va[c] = Jb[(1 + c) * NQ + 3 + a] - Jb[3 + a] * o[c];
                        acc += euler_dd_form(cs, a, bq, cb, va);
                    }
                    qbar[3 + bq] += acc;
                }
            }
            // stage part of the cotangent of y^{k+1}: lambda rows a_k.rbar_R,
            // mu rows d'_l rbar_0 + c_l.rho, gamma rbar_0 (rho world frame)
            float rho[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = cbb[r];
#pragma unroll
                for (int c = 0; c < DIM; ++c) acc += ps.R[r * DIM + c] * rbar[1 + c];
                rho[r] = acc;
            }

            // ---- (b) pair QP: dual optimality system on the free set ----
            float H[NV * NV], rhs[NV], zb[NV];
#pragma unroll
            for (int i = 0; i < NV * NV; ++i) H[i] = 0.f;
#pragma unroll
            for (int i = 0; i < D1; ++i) H[i * NV + i] = 1.f;
            rhs[0] = 1.f + zeta;
#pragma unroll
            for (int r = 0; r < DIM; ++r) rhs[1 + r] = xi[r];
            rhs[DIM + 1] = 1.f;
#pragma unroll
            for (int i = 0; i < NV; ++i) zb[i] = 0.f;
            for (int k = 0; k < nr; ++k) {
                const float y1 = yn[(size_t)k * N];
                if (y1 > 0.f) {
                    const float4 f = rf[k];
                    float wv[NV];
                    wv[0] = 0.f;
                    wv[1] = f.x;
                    wv[2] = f.y;
                    if (DIM == 3) wv[DIM] = f.z;
                    wv[DIM + 1] = -f.w;
                    const float Dk = f.x * f.x + f.y * f.y + (DIM == 3 ? f.z * f.z : 0.f);
                    const float sl = 1.f / (eps * Dk);
                    const float ybar = yb[(size_t)k * N] + dot3<DIM>(f, rbar + 1);
                    const float yh = yk[(size_t)k * N];
#pragma unroll
                    for (int i = 0; i < NV; ++i) {
#pragma unroll
                        for (int j = 0; j < NV; ++j) H[i * NV + j] += sl * wv[i] * wv[j];
                        rhs[i] += yh * wv[i];
                        zb[i] -= ybar * sl * wv[i];
                    }
                }
            }
            // mu rows in world coordinates omega = (d', c); E = diag(1, R^T)
            float M[D1 * D1], mr[D1], mz[D1], cbk[DIM] = {};
#pragma unroll
            for (int i = 0; i < D1 * D1; ++i) M[i] = 0.f;
#pragma unroll
            for (int i = 0; i < D1; ++i) mr[i] = mz[i] = 0.f;
            for (int l = 0; l < no; ++l) {
                const float4 f = of[l];
                const float yh = yk[(size_t)(nr + l) * N];
                cbk[0] += yh * f.x;
                cbk[1] += yh * f.y;
                if (DIM == 3) cbk[DIM - 1] += yh * f.z;
                const float y1 = yn[(size_t)(nr + l) * N];
                if (y1 > 0.f) {
                    const float dp = face_offset(dl, l, f, cl[l], ps.pos64, ps.pos, DIM);
                    float om[D1];
                    om[0] = dp;
                    om[1] = f.x;
                    om[2] = f.y;
                    if (DIM == 3) om[DIM] = f.z;
                    const float Dl = dp * dp + f.x * f.x + f.y * f.y + (DIM == 3 ? f.z * f.z : 0.f);
                    const float sl = 1.f / (eps * Dl);
                    const float ybar = yb[(size_t)(nr + l) * N] + dp * rbar[0] + dot3<DIM>(f, rho);
#pragma unroll
                    for (int i = 0; i < D1; ++i) {
#pragma unroll
                        for (int j = 0; j < D1; ++j) M[i * D1 + j] += sl * om[i] * om[j];
                        mr[i] += yh * om[i];
                        mz[i] -= ybar * sl * om[i];
                    }
                }
            }
            {
                const float y1 = yn[(size_t)(nr + no) * N];
                if (y1 > 0.f) {
                    const float sl = 1.f / eps;
                    H[0] += sl;
                    rhs[0] += yk[(size_t)(nr + no) * N];
                    zb[0] -= (yb[(size_t)(nr + no) * N] + rbar[0]) * sl;
                }
            }
            {
                // E M E^T, E mr, E mz into the first dim+1 coordinates
                float EM[D1 * D1];
#pragma unroll
                for (int j = 0; j < D1; ++j) {
                    EM[j] = M[j];
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        float acc = 0.f;
#pragma unroll
                        for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * M[(1 + m) * D1 + j];
                        EM[(1 + r) * D1 + j] = acc;
                    }
                }
#pragma unroll
                for (int i = 0; i < D1; ++i) {
                    H[i * NV] += EM[i * D1];
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        float acc = 0.f;
#pragma unroll
                        for (int m = 0; m < DIM; ++m) acc += EM[i * D1 + 1 + m] * ps.R[m * DIM + r];
                        H[i * NV + 1 + r] += acc;
                    }
                }
                rhs[0] += mr[0];
                zb[0] += mz[0];
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    float a1 = 0.f, a2 = 0.f;
#pragma unroll
                    for (int m = 0; m < DIM; ++m) {
                        a1 += ps.R[m * DIM + r] * mr[1 + m];
                        a2 += ps.R[m * DIM + r] * mz[1 + m];
                    }
                    rhs[1 + r] += a1;
                    zb[1 + r] += a2;
                }
            }
            float z[NV], ab[NV];
            {
                float Hc[NV * NV];
#pragma unroll
                for (int i = 0; i < NV * NV; ++i) Hc[i] = H[i];
#pragma unroll
                for (int i = 0; i < NV; ++i) z[i] = rhs[i];
                chol_solve<NV>(Hc, z);
#pragma unroll
                for (int i = 0; i < NV; ++i) ab[i] = zb[i];
                chol_solve<NV>(H, ab);
            }
            // cotangents of zeta^k, xi^k: identity part + stage + bhat
            const float tb = zb_in + rbar[0] + ab[0];
            float rb[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) rb[r] = xib_in[r] + rbar[1 + r] + ab[1 + r];
            if (act) {
                A.zb[pr] = tb;
#pragma unroll
                for (int r = 0; r < DIM; ++r) A.xib[((size_t)b * DIM + r) * N + tc - 1] = rb[r];
            }
            float Ra[DIM], Rz[DIM], Rrb[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    a1 += ps.R[r * DIM + c] * ab[1 + c];
                    a2 += ps.R[r * DIM + c] * z[1 + c];
                    a3 += ps.R[r * DIM + c] * rb[c];
                }
                Ra[r] = a1; Rz[r] = a2; Rrb[r] = a3;
            }
            const bool mult = A.has_mult != 0;

            // ---- (c) rows: cotangent of y^k, offsets, pose accumulators ----
            for (int k = 0; k < nr; ++k) {
                const float4 f = rf[k];
                const float y1 = yn[(size_t)k * N];
                float g = 0.f;
                if (y1 > 0.f) g = yb[(size_t)k * N] + dot3<DIM>(f, rbar + 1) + dot3<DIM>(f, ab + 1) - f.w * ab[DIM + 1];
                if (mult) g += dot3<DIM>(f, rb);
                if (act) yb[(size_t)k * N] = g;
            }
            float cb0[DIM] = {}, u2[DIM] = {}, Mcc[DIM * DIM];
#pragma unroll
            for (int i = 0; i < DIM * DIM; ++i) Mcc[i] = 0.f;
            double* gd = A.gdb + (size_t)part * A.n_obs_faces + fo0;
            for (int l = 0; l < no; ++l) {
                const float4 f = of[l];
                const float c3[3] = {f.x, f.y, f.z};
                const float y1 = yn[(size_t)(nr + l) * N];
                const float yh = yk[(size_t)(nr + l) * N];
                const float dp = face_offset(dl, l, f, cl[l], ps.pos64, ps.pos, DIM);
                float dbar = y1 * rbar[0] + (mult ? yh * tb : 0.f);
                float g = 0.f;
                if (y1 > 0.f) {
                    const float ybar = yb[(size_t)(nr + l) * N] + dp * rbar[0] + dot3<DIM>(f, rho);
                    const float Dl = dp * dp + f.x * f.x + f.y * f.y + (DIM == 3 ? f.z * f.z : 0.f);
                    const float sl = 1.f / (eps * Dl);
                    g = ybar + dp * ab[0] + dot3<DIM>(f, Ra);
                    const float p = dp * z[0] + dot3<DIM>(f, Rz);
                    const float Db = p * g * sl / Dl;          // -sbar s / D with sbar = -p g
                    const float K0 = y1 * ab[0] - sl * g * z[0] + 2.f * Db * dp;
                    dbar += K0;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        cb0[r] += K0 * c3[r];
                        u2[r] += sl * g * c3[r];
#pragma unroll
                        for (int m = 0; m < DIM; ++m) Mcc[r * DIM + m] += 2.f * Db * c3[r] * c3[m];
                    }
                }
                if (mult) g += dp * tb + dot3<DIM>(f, Rrb);
                if (act) yb[(size_t)(nr + l) * N] = g;
                const float dsum = wave_sum(act ? dbar : 0.f);
                if (lane == 0) gd[l] += (double)dsum;
            }
            {
                const float y1 = yn[(size_t)(nr + no) * N];
                float g = 0.f;
                if (y1 > 0.f) g = yb[(size_t)(nr + no) * N] + rbar[0] + ab[0];
                if (mult) g += tb;
                if (act) yb[(size_t)(nr + no) * N] = g;
            }
            // pose cotangent of the pair QP: Rbar = cbar abar_R^T - u2 z_R^T
            // + Mcc R - cb0 o^T (the last from pos = rho + R o), pos_bar = -cb0
            {
                float Rb[DIM * DIM];
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int m = 0; m < DIM; ++m) {
                        float acc = cb[r] * ab[1 + m] - u2[r] * z[1 + m] - cb0[r] * o[m];
#pragma unroll
                        for (int q = 0; q < DIM; ++q) acc += Mcc[r * DIM + q] * ps.R[q * DIM + m];
                        Rb[r * DIM + m] = acc;
                    }
#pragma unroll
                for (int r = 0; r < DIM; ++r) qbar[r] -= cb0[r];
#pragma unroll
                for (int a = 0; a < NATT; ++a) {
                    float acc = 0.f;
#pragma unroll
                    for (int i = 0; i < DIM * DIM; ++i) acc += Rb[i] * ps.dR[a * DIM * DIM + i];
                    qbar[DIM + a] += acc;
                }
            }
            // multiplier update of the previous step at (x^k, y^k): J^T (tb, rb)
            if (mult) {
                pair_jacobian<DIM>(ps, cbk, o, J);
#pragma unroll
                for (int a = 0; a < NQ; ++a) {
                    float acc = J[a] * tb;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) acc += J[(1 + r) * NQ + a] * rb[r];
                    qbar[a] += acc;
                }
            }
        }
        // workgroup sum of the pose cotangents (fixed order over the waves)
#pragma unroll
        for (int a = 0; a < NQ; ++a) red[(wave * NQ + a) * 64 + lane] = act ? qbar[a] : 0.f;
        __syncthreads();
        float* out = A.qpart + (size_t)wg * NQ * 64;
        for (int e = threadIdx.x; e < NQ * 64; e += blockDim.x) {
            float acc = 0.f;
            for (int w = 0; w < W; ++w) acc += red[w * NQ * 64 + e];
            out[e] = acc;
        }
        __syncthreads();
    }
}

// grad_d[f] = scale * sum_i gdb[i][f]; grad_x0 = scale * gx0
__global__ void grad_finalize_kernel(int n_parts, int n_faces, const double* gdb, int n_x0, const double* gx0,
                                     float scale, float* grad_d, float* grad_x0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_faces) {
        double acc = 0.0;
        for (int p = 0; p < n_parts; ++p) acc += gdb[(size_t)p * n_faces + i];
        grad_d[i] = (float)(scale * acc);
    }
    if (i < n_x0) grad_x0[i] = (float)(scale * gx0[i]);
}

hipError_t launch_pair_adjoint(const DevProblem& P, const PairAdjoint& A, int W, int grid, hipStream_t st)
{
    if (P.n_blocks == 0) return hipSuccess;
    dim3 blk(64 * W), grd(grid);
    const size_t slot = sizeof(float4) * (CADMM_MAX_PART_FACES + CADMM_MAX_OBS_FACES) +
                        sizeof(double) * CADMM_MAX_OBS_FACES;
    if (P.dim == 2)
        hipLaunchKernelGGL(pair_adjoint_kernel<2>, grd, blk, W * slot + sizeof(float) * W * Pose<2>::NQ * 64, st, P,
                           A);
    else
        hipLaunchKernelGGL(pair_adjoint_kernel<3>, grd, blk, W * slot + sizeof(float) * W * Pose<3>::NQ * 64, st, P,
                           A);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(int n_parts, int n_faces, const double* gdb, int n_x0, const double* gx0,
                                float scale, float* grad_d, float* grad_x0, hipStream_t st)
{
    const int n = n_faces > n_x0 ? n_faces : n_x0;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(grad_finalize_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n_parts, n_faces, gdb, n_x0,
                       gx0, scale, grad_d, grad_x0);
    return hipGetLastError();
}

}  // namespace cadmm
