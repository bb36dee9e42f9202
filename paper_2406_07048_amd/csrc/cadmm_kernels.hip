// gfx950 kernels of the ADMM collision-avoidance path (arXiv 2406.07048).
//
// Work decomposition (one wavefront = one pair block):
//   a pair block is (scenario s, robot part i, obstacle j) with its N pairs
//   t = 1..N; lane t-1 of the wave owns pair (i, j, t). The block's geometry
//   (faces of part i and obstacle j) is wave-uniform and is read through the
//   scalar cache; each lane keeps its pair's small QP in registers.
//   A workgroup holds up to 8 waves = blocks of the same scenario, so the
//   per-time-step sums of the trajectory-QP contributions are formed in LDS
//   (fixed order, no float atomics) and written once per workgroup.
//
// Numerics: FP32 throughout. The dual-update QP is solved in its (dim+2)-
// dimensional dual (residual v = K^T y + bhat and the multiplier nu of the
// equality) by a semismooth Newton method with an exact-sign line search;
// the primal y is recovered row by row as max(0, yhat - (K_l v - kappa_l nu)
// / (eps D_l)).
#include "cadmm_device.h"

#include <float.h>
#include <math.h>

namespace cadmm {


// ------------------------------------------------------------------------
// the pair sub-problem in the ADMM kernel: structured rows
//   lambda rows k: K_k = (0, a_k), kappa_k = b_k
//   mu rows l:     K_l = (d'_l, R^T c_l), d'_l = d_l - c_l.pos, kappa_l = 0
//   gamma row:     K = (1, 0), kappa = 0
// Each lane keeps d'_l of its rows (small near the obstacle, so no
// cancellation against the world-frame offsets); the obstacle normals c_l
// come from the block's LDS copy. Slopes use s_l = d'_l v0 + c_l.(R v_r), and
// the mu-row Hessian block is E M E^T with E = diag(1, R^T) and
// M = sum f (d', c)(d', c)^T.
// A pair is solved by a group of G lanes (G = 1, 2, 4): lane q of the group
// owns the lambda and mu rows with index = q (mod G) and the group sums its
// partial sums with group_sum, so every lane of the group holds the same
// Newton iterate. The gamma row is evaluated by every lane and counted once.
// ------------------------------------------------------------------------

template <int DIM, int MR, int MO, int G>
struct PairRows {
    static constexpr int NV = DIM + 2;
    static constexpr int RR = (MR + G - 1) / G;   // lambda rows per lane
    static constexpr int RO = (MO + G - 1) / G;   // mu rows per lane
    int q;                     // lane within the group
    int nr, no;
    const float4* rf;          // robot faces of the part (LDS)
    const float4* of;          // obstacle faces (LDS)
    float R[DIM * DIM];
    float bh[DIM + 1];
    float yhR[RR], yhO[RO], yhG;
    float ieR[RR], ieO[RO], ieG;    // 1 / (eps D_l)
    float dpO[RO];                  // d'_l of the pair

    template <bool HESS>
    __device__ __forceinline__ void pass(const float (&z)[NV], float (&g)[NV], float (&H)[NV * NV],
                                         float& sc) const
    {
        const float v0 = z[0], nu = z[DIM + 1];
        float vr[DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r) vr[r] = z[1 + r];
        float w[DIM];   // R v_r
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            float acc = 0.f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc += R[r * DIM + c] * vr[c];
            w[r] = acc;
        }
        // partial sums of this lane's rows
        constexpr int NH = DIM * (DIM + 1) / 2;          // lambda-row Hessian block (upper)
        constexpr int NM = (DIM + 1) * (DIM + 2) / 2;    // mu-row (d', c) moments (upper)
        float gl[DIM] = {}, gnu = 0.f, Sd = 0.f, Sc[DIM] = {}, ysc = 0.f;
        float Hl[NH] = {}, Hln[DIM] = {}, Hnn = 0.f, M[NM] = {};
#pragma unroll
        for (int m = 0; m < RR; ++m) {
            const int k = q + G * m;
            if (k < nr) {
                const float4 f = rf[k];
                const float a[3] = {f.x, f.y, f.z};
                float s = -f.w * nu, an = 0.f;
#pragma unroll
                for (int r = 0; r < DIM; ++r) { s += a[r] * vr[r]; an += fabsf(a[r]); }
                const float y = fmaxf(0.f, yhR[m] - s * ieR[m]);
#pragma unroll
                for (int r = 0; r < DIM; ++r) gl[r] += y * a[r];
                gnu += f.w * y;
                ysc += y * an;
                if (HESS) {
                    const float act = y > 0.f ? ieR[m] : 0.f;
                    int h = 0;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
#pragma unroll
                        for (int c = r; c < DIM; ++c) Hl[h++] += act * a[r] * a[c];
                        Hln[r] += act * f.w * a[r];
                    }
                    Hnn += act * f.w * f.w;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < RO; ++m) {
            const int l = q + G * m;
            if (l < no) {
                const float4 f = of[l];
                const float ch[4] = {dpO[m], f.x, f.y, f.z};   // (d'_l, c_l)
                float s = ch[0] * v0, cn = 0.f;
#pragma unroll
                for (int r = 0; r < DIM; ++r) { s += ch[1 + r] * w[r]; cn += fabsf(ch[1 + r]); }
                const float y = fmaxf(0.f, yhO[m] - s * ieO[m]);
                Sd += ch[0] * y;
#pragma unroll
                for (int r = 0; r < DIM; ++r) Sc[r] += ch[1 + r] * y;
                ysc += y * (fabsf(ch[0]) + cn);
                if (HESS) {
                    const float act = y > 0.f ? ieO[m] : 0.f;
                    int h = 0;
#pragma unroll
                    for (int r = 0; r <= DIM; ++r)
#pragma unroll
                        for (int c = r; c <= DIM; ++c) M[h++] += act * ch[r] * ch[c];
                }
            }
        }
        // group sums (every lane of the group gets the same values)
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            gl[r] = group_sum<G>(gl[r]);
            Sc[r] = group_sum<G>(Sc[r]);
        }
        gnu = group_sum<G>(gnu);
        Sd = group_sum<G>(Sd);
        ysc = group_sum<G>(ysc);
        if (HESS) {
#pragma unroll
            for (int h = 0; h < NH; ++h) Hl[h] = group_sum<G>(Hl[h]);
#pragma unroll
            for (int r = 0; r < DIM; ++r) Hln[r] = group_sum<G>(Hln[r]);
            Hnn = group_sum<G>(Hnn);
#pragma unroll
            for (int h = 0; h < NM; ++h) M[h] = group_sum<G>(M[h]);
        }
        const float yg = fmaxf(0.f, yhG - v0 * ieG);
        ysc += yg;
        // gradient of the dual function
        g[0] = bh[0] - v0 + Sd + yg;
#pragma unroll
        for (int r = 0; r < DIM; ++r) {
            float acc = 0.f;
#pragma unroll
            for (int m = 0; m < DIM; ++m) acc += R[m * DIM + r] * Sc[m];
            g[1 + r] = bh[1 + r] - vr[r] + gl[r] + acc;
        }
        g[DIM + 1] = 1.f - gnu;
        float mx = fabsf(v0);
#pragma unroll
        for (int r = 0; r < DIM; ++r) mx = fmaxf(mx, fabsf(vr[r]));
        float bm = fabsf(bh[0]);
#pragma unroll
        for (int r = 0; r < DIM; ++r) bm = fmaxf(bm, fabsf(bh[1 + r]));
        sc = 1.f + bm + mx + ysc;
        if (HESS) {
            // full symmetric (d', c) moment matrix and lambda block
            float Mf[(DIM + 1) * (DIM + 1)], Hf[DIM * DIM];
            {
                int h = 0;
#pragma unroll
                for (int r = 0; r <= DIM; ++r)
#pragma unroll
                    for (int c = r; c <= DIM; ++c) {
                        Mf[r * (DIM + 1) + c] = M[h];
                        Mf[c * (DIM + 1) + r] = M[h];
                        ++h;
                    }
                h = 0;
#pragma unroll
                for (int r = 0; r < DIM; ++r)
#pragma unroll
                    for (int c = r; c < DIM; ++c) {
                        Hf[r * DIM + c] = Hl[h];
                        Hf[c * DIM + r] = Hl[h];
                        ++h;
                    }
            }
            // H_vv = I + diag(1, R^T) M diag(1, R)  (+ lambda and gamma rows)
            float MR_[(DIM + 1) * DIM];   // M[:, 1:] R  -> (DIM+1) x DIM
#pragma unroll
            for (int r = 0; r <= DIM; ++r)
#pragma unroll
                for (int qq = 0; qq < DIM; ++qq) {
                    float acc = 0.f;
#pragma unroll
                    for (int e = 0; e < DIM; ++e) acc += Mf[r * (DIM + 1) + 1 + e] * R[e * DIM + qq];
                    MR_[r * DIM + qq] = acc;
                }
            H[0] = Mf[0] + 1.f + (yg > 0.f ? ieG : 0.f);
#pragma unroll
            for (int qq = 0; qq < DIM; ++qq) H[1 + qq] = MR_[qq];
#pragma unroll
            for (int r = 0; r < DIM; ++r)
#pragma unroll
                for (int qq = r; qq < DIM; ++qq) {
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) acc += R[c * DIM + r] * MR_[(1 + c) * DIM + qq];
                    H[(1 + r) * NV + 1 + qq] = acc + (r == qq ? 1.f : 0.f) + Hf[r * DIM + qq];
                }
#pragma unroll
            for (int r = 0; r < DIM; ++r) H[(1 + r) * NV + DIM + 1] = -Hln[r];
            H[0 * NV + DIM + 1] = 0.f;
            H[(DIM + 1) * NV + DIM + 1] = Hnn + 1e-6f * (1.f + Hnn);
#pragma unroll
            for (int r = 0; r < NV; ++r)
#pragma unroll
                for (int c = 0; c < r; ++c) H[r * NV + c] = H[c * NV + r];
        }
    }
};

// ------------------------------------------------------------------------
// generic rows (stateless batch entry point): K, kappa, yhat from memory
// ------------------------------------------------------------------------

template <int DIM>
struct GenRows {
    static constexpr int NV = DIM + 2;
    int n;
    const float* K;
    const float* kap;
    const float* yh;
    float eps;
    float bh[DIM + 1];

    template <bool HESS>
    __device__ __forceinline__ void pass(const float (&z)[NV], float (&g)[NV], float (&H)[NV * NV],
                                         float& sc) const
    {
        float gv[DIM + 1] = {}, gnu = 0.f, ysc = 0.f;
        if (HESS) {
#pragma unroll
            for (int i = 0; i < NV * NV; ++i) H[i] = 0.f;
        }
        for (int l = 0; l < n; ++l) {
            float k[DIM + 1];
            float D = 0.f;
#pragma unroll
            for (int c = 0; c <= DIM; ++c) { k[c] = K[l * (DIM + 1) + c]; D += k[c] * k[c]; }
            const float kl = kap[l];
            const float ie = 1.0f / (eps * D);
            float s = -kl * z[DIM + 1];
#pragma unroll
            for (int c = 0; c <= DIM; ++c) s += k[c] * z[c];
            const float y = fmaxf(0.f, yh[l] - s * ie);
#pragma unroll
            for (int c = 0; c <= DIM; ++c) gv[c] += y * k[c];
            gnu += kl * y;
            ysc += y * sqrtf(D);
            if (HESS && y > 0.f) {
                float w[NV];
#pragma unroll
                for (int c = 0; c <= DIM; ++c) w[c] = k[c];
                w[DIM + 1] = -kl;
#pragma unroll
                for (int r = 0; r < NV; ++r)
#pragma unroll
                    for (int c = r; c < NV; ++c) H[r * NV + c] += ie * w[r] * w[c];
            }
        }
        float mx = 0.f, bm = 0.f;
#pragma unroll
        for (int c = 0; c <= DIM; ++c) {
            g[c] = bh[c] - z[c] + gv[c];
            mx = fmaxf(mx, fabsf(z[c]));
            bm = fmaxf(bm, fabsf(bh[c]));
        }
        g[DIM + 1] = 1.f - gnu;
        sc = 1.f + bm + mx + ysc;
        if (HESS) {
#pragma unroll
            for (int c = 0; c <= DIM; ++c) H[c * NV + c] += 1.f;
            H[(DIM + 1) * NV + DIM + 1] += 1e-6f * (1.f + H[(DIM + 1) * NV + DIM + 1]);
#pragma unroll
            for (int r = 0; r < NV; ++r)
#pragma unroll
                for (int c = 0; c < r; ++c) H[r * NV + c] = H[c * NV + r];
        }
    }
};

// ------------------------------------------------------------------------
// semismooth Newton on the concave dual, shared by both row sources.
// Returns the sweeps used, or -1 if the budget ran out (z is still the last
// iterate, whose primal y is within the Newton region in practice).
// ------------------------------------------------------------------------

template <int NV, class Rows>
__device__ int dual_newton(const Rows& rows, float (&z)[NV], int max_sweeps)
{
    float gprev = FLT_MAX;
    float al_prev = 1.f;   // step accepted by the previous sweep
    for (int it = 0; it < max_sweeps; ++it) {
        float g[NV], H[NV * NV], sc;
        rows.template pass<true>(z, g, H, sc);
        float gmax = 0.f, zmax = 0.f;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            gmax = fmaxf(gmax, fabsf(g[i]));
            zmax = fmaxf(zmax, fabsf(z[i]));
        }
        // converged, or stalled at the rounding floor of the gradient. On C3
        // pairs (FP32 against the FP64 active-set solution) every iterate with
        // gmax <= 1e-6 sc had a scaled dual error <= 3.4e-6, and iterates that
        // stop improving below 4e-6 sc sit at the FP32 floor of the gradient
        // (error <= 7e-6); iterating on there only spent the sweep budget.
        if (gmax <= 1e-6f * sc || (gmax <= 4e-6f * sc && gmax >= 0.7f * gprev)) return it;
        gprev = gmax;
        float dz[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) dz[i] = g[i];
        chol_solve<NV>(H, dz);
        // After a short step the direction is often steered by rows whose
        // dual is about to reach zero; they stop it at the first kink every
        // sweep. Re-solve with the generalised Hessian of the active set at
        // the full step (a primal-dual active-set correction) and take that
        // direction when it is still an ascent direction.
        if (al_prev < 0.1f) {
            float zt[NV], gt[NV], Ht[NV * NV], sct, dz2[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) zt[i] = z[i] + dz[i];
            rows.template pass<true>(zt, gt, Ht, sct);
#pragma unroll
            for (int i = 0; i < NV; ++i) dz2[i] = g[i];
            chol_solve<NV>(Ht, dz2);
            float e0 = 0.f;
#pragma unroll
            for (int i = 0; i < NV; ++i) e0 += dz2[i] * g[i];
            if (e0 > 0.f) {
#pragma unroll
                for (int i = 0; i < NV; ++i) dz[i] = dz2[i];
            }
        }
        // Newton step at the rounding level of z: the active set is settled
        // and z is the optimum to working precision
        float dmax = 0.f;
#pragma unroll
        for (int i = 0; i < NV; ++i) dmax = fmaxf(dmax, fabsf(dz[i]));
        if (dmax <= 1e-6f * (zmax + 1e-3f * sc)) {
#pragma unroll
            for (int i = 0; i < NV; ++i) z[i] += dz[i];
            return it + 1;
        }
        float d0 = 0.f;
#pragma unroll
        for (int i = 0; i < NV; ++i) d0 += dz[i] * g[i];
        if (!(d0 > 0.f)) return it;
        // directional derivative of the dual along dz at step al
        auto dphi = [&](float al) {
            float zt[NV], gt[NV], Hd[NV * NV], sct;
#pragma unroll
            for (int i = 0; i < NV; ++i) zt[i] = z[i] + al * dz[i];
            rows.template pass<false>(zt, gt, Hd, sct);
            float d = 0.f;
#pragma unroll
            for (int i = 0; i < NV; ++i) d += dz[i] * gt[i];
            return d;
        };
        float al = 1.f;
        const float d1 = dphi(1.f);
        if (d1 < -1e-3f * d0) {
            // Illinois regula falsi on the decreasing piecewise-linear dphi
            float lo = 0.f, hi = 1.f, flo = d0, fhi = d1;
            int side = 0;
            for (int ls = 0; ls < 6; ++ls) {
                al = (lo * (-fhi) + hi * flo) / (flo - fhi);
                const float fa = dphi(al);
                if (fa >= -1e-3f * d0) {
                    lo = al; flo = fa;
                    if (side == 1) fhi *= 0.5f;
                    side = 1;
                    if (fa <= 0.1f * d0) break;
                } else {
                    hi = al; fhi = fa;
                    if (side == -1) flo *= 0.5f;
                    side = -1;
                }
            }
            al = lo;
            // no step along dz passes the test: at the FP32 floor of the
            // directional derivative z cannot be improved, and every further
            // sweep would repeat this one exactly
            if (al == 0.f) return it + 1;
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) z[i] += al * dz[i];
        al_prev = al;
    }
    return -1;
}

// ------------------------------------------------------------------------
// ADMM step 1: dual updates of every pair + linearised contributions
// ------------------------------------------------------------------------

template <int DIM>
struct Contrib {
    static constexpr int NQ = Pose<DIM>::NQ;
    static constexpr int NC = NQ * (NQ + 1) / 2 + NQ;
};

// Arg-max of (value, payload) over a lane group with ties to the smaller
// key; every lane of the group ends with the same triple.
template <int G>
__device__ __forceinline__ void group_argmax(float& v, float& pay, int& key)
{
    if constexpr (G >= 2) {
        const float ov = dpp_xor1(v), op = dpp_xor1(pay);
        const int ok = dpp_xor1_i(key);
        if (ov > v || (ov == v && ok < key)) { v = ov; pay = op; key = ok; }
    }
    if constexpr (G >= 4) {
        const float ov = dpp_xor2(v), op = dpp_xor2(pay);
        const int ok = dpp_xor2_i(key);
        if (ov > v || (ov == v && ok < key)) { v = ov; pay = op; key = ok; }
    }
}

// Waves per pair block: a wave holds 64 / G pairs.
__host__ __device__ constexpr int pair_waves_per_block(int N, int G)
{
    return (N + 64 / G - 1) / (64 / G);
}

// One workgroup = WB pair blocks of one scenario, each spread over
// pair_waves_per_block(N, G) waves; lane L of a block's wave c solves pair
// t = c * (64 / G) + L / G + 1 with its group lane q = L % G.
template <int DIM, int MR, int MO, int G>
__global__ void __launch_bounds__(512) pair_phase_kernel(DevProblem P)
{
    constexpr int NV = DIM + 2;
    constexpr int NATT = Pose<DIM>::NATT;
    constexpr int NQ = Pose<DIM>::NQ;
    constexpr int NC = Contrib<DIM>::NC;
    constexpr int PPW = 64 / G;                    // pairs per wave
    using Rows = PairRows<DIM, MR, MO, G>;
    extern __shared__ __align__(16) float lds[];
    const int N = P.N;
    const int nw = pair_waves_per_block(N, G);
    const int W = blockDim.x >> 6;                 // waves in the workgroup
    const int WB = W / nw;                         // blocks in the workgroup
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int bslot = wave / nw, chunk = wave % nw;
    const int q = lane % G;
    const int t = chunk * PPW + lane / G + 1;
    float4* faces = reinterpret_cast<float4*>(lds);   // [WB][MR + MO] faces of each block
    float* red = lds + 4 * WB * (MR + MO);            // [WB][NC][64] contributions by step
    float* red_rd = red + WB * NC * 64;               // [W]
    int* red_un = reinterpret_cast<int*>(red_rd + W);
    const float eps = P.eps_prox;

    for (int wg = blockIdx.x; wg < P.n_wg; wg += gridDim.x) {
        const int4 item = P.wg_items[wg];
        const int s = uniform(item.x);
        if (P.done[s]) continue;                 // uniform over the workgroup
        const int b = uniform(item.y + bslot);
        // the block's faces into its LDS slot: every solver pass reads them,
        // and from LDS they are cheap reads instead of HBM round trips
        float4* fl = faces + bslot * (MR + MO);
        if (b < item.z && chunk == 0) {
            const int4 bk = P.blocks[b];
            const int f0 = P.part_face_ptr[bk.y], nf = P.part_face_ptr[bk.y + 1] - f0;
            const int g0 = P.obs_face_ptr[bk.z], ng = P.obs_face_ptr[bk.z + 1] - g0;
            if (lane < nf) fl[lane] = P.part_faces[f0 + lane];
            else if (lane >= MR && lane - MR < ng) fl[lane] = P.obs_faces[g0 + lane - MR];
        }
        __syncthreads();
        float con[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) con[c] = 0.f;
        float rd = 0.f;
        int unc = 0;
        if (b < item.z && t <= N) {
            const int4 blk = P.blocks[b];
            const int part = uniform(blk.y), obs = uniform(blk.z);
            const int fr0 = uniform(P.part_face_ptr[part]);
            const int fo0 = uniform(P.obs_face_ptr[obs]);
            Rows pr;
            pr.q = q;
            pr.nr = uniform(P.part_face_ptr[part + 1] - fr0);
            pr.no = uniform(P.obs_face_ptr[obs + 1] - fo0);
            pr.rf = fl;
            pr.of = fl + MR;
            const int yoff = uniform(P.block_yoff[b]);
            const float* xs = P.x + ((size_t)s * (N + 1) + t) * P.n_s;
            Pose<DIM> ps;
            make_pose<DIM>(P, xs, part, ps);
#pragma unroll
            for (int i = 0; i < DIM * DIM; ++i) pr.R[i] = ps.R[i];
            const float zeta = P.zeta[(size_t)b * N + t - 1];
            float xi[DIM];
#pragma unroll
            for (int r = 0; r < DIM; ++r) xi[r] = P.xi[((size_t)b * DIM + r) * N + t - 1];
            pr.bh[0] = 1.f + zeta;
#pragma unroll
            for (int r = 0; r < DIM; ++r) pr.bh[1 + r] = xi[r];
            const float* yb = P.y + yoff + (t - 1);
            // warm start v = K^T yhat + bhat, nu from the largest lambda row
            float v0 = 0.f, Sc[DIM] = {}, vr[DIM] = {};
#pragma unroll
            for (int m = 0; m < Rows::RR; ++m) {
                const int k = q + G * m;
                if (k < pr.nr) {
                    const float4 f = pr.rf[k];
                    const float yk = yb[k * N];
                    pr.yhR[m] = yk;
                    const float D = f.x * f.x + f.y * f.y + (DIM == 3 ? f.z * f.z : 0.f);
                    pr.ieR[m] = 1.0f / (eps * D);
                    vr[0] += yk * f.x;
                    vr[1] += yk * f.y;
                    if (DIM == 3) vr[DIM - 1] += yk * f.z;
                } else {
                    pr.yhR[m] = 0.f; pr.ieR[m] = 0.f;
                }
            }
#pragma unroll
            for (int m = 0; m < Rows::RO; ++m) {
                const int l = q + G * m;
                if (l < pr.no) {
                    const float4 f = pr.of[l];
                    const float c[3] = {f.x, f.y, f.z};
                    const float yl = yb[(pr.nr + l) * N];
                    pr.yhO[m] = yl;
                    const float dp = face_offset(P.obs_d64, fo0 + l, f, ps.pos64, DIM);
                    float cn = 0.f;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) cn += c[r] * c[r];
                    const float D = dp * dp + cn;
                    pr.ieO[m] = 1.0f / (eps * D);
                    pr.dpO[m] = dp;
                    v0 += dp * yl;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) Sc[r] += c[r] * yl;
                } else {
                    pr.yhO[m] = 0.f; pr.ieO[m] = 0.f; pr.dpO[m] = 0.f;
                }
            }
            v0 = group_sum<G>(v0);
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                vr[r] = group_sum<G>(vr[r]);
                Sc[r] = group_sum<G>(Sc[r]);
            }
            pr.yhG = yb[(pr.nr + pr.no) * N];
            pr.ieG = 1.0f / eps;
            v0 += pr.bh[0] + pr.yhG;
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * Sc[m];
                vr[r] += pr.bh[1 + r] + acc;
            }
            float best = -1.f, nu = 0.f;
            int kbest = 1 << 30;
#pragma unroll
            for (int m = 0; m < Rows::RR; ++m) {
                const int k = q + G * m;
                if (k < pr.nr && pr.yhR[m] > best) {
                    const float4 f = pr.rf[k];
                    best = pr.yhR[m];
                    kbest = k;
                    nu = (f.x * vr[0] + f.y * vr[1] + (DIM == 3 ? f.z * vr[DIM - 1] : 0.f)) / f.w;
                }
            }
            group_argmax<G>(best, nu, kbest);
            float z[NV];
            z[0] = v0;
#pragma unroll
            for (int r = 0; r < DIM; ++r) z[1 + r] = vr[r];
            z[DIM + 1] = nu;
            const int sweeps = dual_newton<NV>(pr, z, P.max_sweeps);
            unc = (sweeps < 0 && q == 0) ? 1 : 0;

            // final pass: primal rows, write-back, residual and Jacobian
            {
                const float zv0 = z[0], znu = z[DIM + 1];
                float w[DIM];
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    float acc = 0.f;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) acc += ps.R[r * DIM + c] * z[1 + c];
                    w[r] = acc;
                }
                float* yw = P.y + yoff + (t - 1);
                float Al[DIM] = {}, Sd = 0.f, Scf[DIM] = {};
#pragma unroll
                for (int m = 0; m < Rows::RR; ++m) {
                    const int k = q + G * m;
                    if (k < pr.nr) {
                        const float4 f = pr.rf[k];
                        float s = -f.w * znu + f.x * z[1] + f.y * z[2] + (DIM == 3 ? f.z * z[DIM] : 0.f);
                        const float y = fmaxf(0.f, pr.yhR[m] - s * pr.ieR[m]);
                        yw[k * N] = y;
                        const float dl = y - pr.yhR[m];
                        rd += dl * dl;
                        Al[0] += y * f.x;
                        Al[1] += y * f.y;
                        if (DIM == 3) Al[DIM - 1] += y * f.z;
                    }
                }
#pragma unroll
                for (int m = 0; m < Rows::RO; ++m) {
                    const int l = q + G * m;
                    if (l < pr.no) {
                        const float4 f = pr.of[l];
                        const float c[3] = {f.x, f.y, f.z};
                        float s = pr.dpO[m] * zv0;
#pragma unroll
                        for (int r = 0; r < DIM; ++r) s += c[r] * w[r];
                        const float y = fmaxf(0.f, pr.yhO[m] - s * pr.ieO[m]);
                        yw[(pr.nr + l) * N] = y;
                        const float dl = y - pr.yhO[m];
                        rd += dl * dl;
                        Sd += pr.dpO[m] * y;
#pragma unroll
                        for (int r = 0; r < DIM; ++r) Scf[r] += c[r] * y;
                    }
                }
                Sd = group_sum<G>(Sd);
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    Al[r] = group_sum<G>(Al[r]);
                    Scf[r] = group_sum<G>(Scf[r]);
                }
                const float yg = fmaxf(0.f, pr.yhG - zv0 * pr.ieG);
                if (q == 0) yw[(pr.nr + pr.no) * N] = yg;   // gamma is not in the dual residual sum
                // residual e = K^T y + bhat at s^k
                float e[DIM + 1];
                e[0] = 1.f + zeta + Sd + yg;
#pragma unroll
                for (int r = 0; r < DIM; ++r) {
                    float acc = Al[r] + xi[r];
#pragma unroll
                    for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * Scf[m];
                    e[1 + r] = acc;
                }
                // Jacobian of (T, R) in the pose coordinates (position, attitude)
                const float* o = P.part_off + part * 3;
                float J[(DIM + 1) * NQ];
#pragma unroll
                for (int i = 0; i < (DIM + 1) * NQ; ++i) J[i] = 0.f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) J[c] = -Scf[c];
#pragma unroll
                for (int a = 0; a < NATT; ++a) {
                    const float* dRa = ps.dR + a * DIM * DIM;
                    float acc = 0.f;
#pragma unroll
                    for (int r = 0; r < DIM; ++r)
#pragma unroll
                        for (int c = 0; c < DIM; ++c) acc += Scf[r] * dRa[r * DIM + c] * o[c];
                    J[DIM + a] = -acc;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) {
                        float v = 0.f;
#pragma unroll
                        for (int m = 0; m < DIM; ++m) v += dRa[m * DIM + r] * Scf[m];
                        J[(1 + r) * NQ + DIM + a] = v;
                    }
                }
                // stage terms in deviation coordinates about x^k (the
                // trajectory QP solves for x - x^k): Hessian sigma J^T J and
                // gradient sigma J^T e, with no -J q^k term to cancel
                const float sg = P.sigma;
                int idx = 0;
#pragma unroll
                for (int i = 0; i < NQ; ++i)
#pragma unroll
                    for (int j = i; j < NQ; ++j) {
                        float acc = 0.f;
#pragma unroll
                        for (int m = 0; m <= DIM; ++m) acc += J[m * NQ + i] * J[m * NQ + j];
                        con[idx++] = sg * acc;
                    }
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    float acc = 0.f;
#pragma unroll
                    for (int m = 0; m <= DIM; ++m) acc += J[m * NQ + i] * e[m];
                    con[idx++] = sg * acc;
                }
            }
        }
        // contributions by step t into the block's slot (lane q = 0 of each
        // group; lanes of empty slots write zeros), then the workgroup sum
        // over its blocks in a fixed order
        const float rdw = wave_sum(rd);
        const int unw = wave_sum_int(unc);
        if (q == 0 && t <= 64) {
#pragma unroll
            for (int c = 0; c < NC; ++c) red[(bslot * NC + c) * 64 + t - 1] = con[c];
        }
        if (lane == 0) { red_rd[wave] = rdw; red_un[wave] = unw; }
        __syncthreads();
        float* out = P.contrib + (size_t)wg * NC * 64;
        for (int e = threadIdx.x; e < NC * 64; e += blockDim.x) {
            float acc = 0.f;
            if ((e & 63) < N)
                for (int w = 0; w < WB; ++w) acc += red[w * NC * 64 + e];
            out[e] = acc;
        }
        if (threadIdx.x == 0) {
            float a = 0.f;
            int u = 0;
            for (int w = 0; w < W; ++w) { a += red_rd[w]; u += red_un[w]; }
            P.rdual_part[wg] = a;
            P.unconv_part[wg] = u;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// ADMM step 3: multiplier update zeta += T(s^{k+1}, y^{k+1}),
// xi += R(s^{k+1}, y^{k+1}) and the primal residual partial sums
// ------------------------------------------------------------------------

template <int DIM, int MR, int MO>
__global__ void __launch_bounds__(512) mult_phase_kernel(DevProblem P)
{
    extern __shared__ float lds[];
    const int W = blockDim.x >> 6;
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int N = P.N;
    for (int wg = blockIdx.x; wg < P.n_wg; wg += gridDim.x) {
        const int4 item = P.wg_items[wg];
        const int s = uniform(item.x);
        if (P.done[s]) continue;
        const int b = uniform(item.y + wave);
        const int t = lane + 1;
        float rp = 0.f;
        if (b < item.z && t <= N) {
            const int4 blk = P.blocks[b];
            const int part = uniform(blk.y), obs = uniform(blk.z);
            const int fr0 = uniform(P.part_face_ptr[part]);
            const int nr = uniform(P.part_face_ptr[part + 1] - fr0);
            const int fo0 = uniform(P.obs_face_ptr[obs]);
            const int no = uniform(P.obs_face_ptr[obs + 1] - fo0);
            const int yoff = uniform(P.block_yoff[b]);
            Pose<DIM> ps;
            make_pose<DIM>(P, P.x + ((size_t)s * (N + 1) + t) * P.n_s, part, ps);
            const float* yb = P.y + yoff + (t - 1);
            float Al[DIM] = {}, Sd = 0.f, Sc[DIM] = {};
#pragma unroll
            for (int k = 0; k < MR; ++k) {
                if (k < nr) {
                    const float4 f = P.part_faces[fr0 + k];
                    const float y = yb[k * N];
                    Al[0] += y * f.x;
                    Al[1] += y * f.y;
                    if (DIM == 3) Al[DIM - 1] += y * f.z;
                }
            }
#pragma unroll
            for (int l = 0; l < MO; ++l) {
                if (l < no) {
                    const float4 f = P.obs_faces[fo0 + l];
                    const float y = yb[(nr + l) * N];
                    const float dp = face_offset(P.obs_d64, fo0 + l, f, ps.pos64, DIM);
                    Sd += dp * y;
                    Sc[0] += f.x * y;
                    Sc[1] += f.y * y;
                    if (DIM == 3) Sc[DIM - 1] += f.z * y;
                }
            }
            const float yg = yb[(nr + no) * N];
            const float T = 1.f + Sd + yg;
            float* zp = P.zeta + (size_t)b * N + t - 1;
            *zp += T;
            rp = T * T;
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = Al[r];
#pragma unroll
                for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * Sc[m];
                P.xi[((size_t)b * DIM + r) * N + t - 1] += acc;
                rp += acc * acc;
            }
        }
        const float rw = wave_sum(rp);
        if (lane == 0) lds[wave] = rw;
        __syncthreads();
        if (threadIdx.x == 0) {
            float a = 0.f;
            for (int w = 0; w < W; ++w) a += lds[w];
            P.rpri_part[wg] = a;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// residual sums, stopping test (Sec. IV-B) and history; one block/scenario
// ------------------------------------------------------------------------

__global__ void __launch_bounds__(64) residual_kernel(DevProblem P)
{
    const int s = blockIdx.x;
    if (P.done[s]) return;
    const int2 r = P.scen_wg[s];
    float a = 0.f, b = 0.f;
    int u = 0;
    for (int w = r.x + threadIdx.x; w < r.y; w += 64) {
        a += P.rpri_part[w];
        b += P.rdual_part[w];
        u += P.unconv_part[w];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    u = wave_sum_int(u);
    if (threadIdx.x == 0) {
        const int k = P.iters[s];
        if (k < P.hist_cap) {
            P.hist_pri[(size_t)k * P.n_scen + s] = a;
            P.hist_dual[(size_t)k * P.n_scen + s] = b;
        }
        P.iters[s] = k + 1;
        P.r_pri[s] = a;
        P.r_dual[s] = b;
        P.unconv[s] = u;
        if (a <= P.eps_pri && b <= P.eps_dual) P.done[s] = 1;
    }
}

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

// Threads of the trajectory kernel: one output per thread in every phase of
// the sweep (512 for the 16/8 padding, 256 otherwise).
__host__ __device__ constexpr int traj_threads(int NS, int NU)
{
    return (NS * NS + NS * NU + NS > 256 || NU * NU + NU * NS + NU + NS * NS + NS > 256) ? 512 : 256;
}

// Floats of the gains region, which first holds the staged trajectory
// (x and x_ref over t = 0..N, u over t = 0..N-1, padded to NS / NU).
__host__ __device__ inline int traj_gain_floats(int N, int NS, int NU)
{
    const int gains = N * NU * (NS + 1), stage = 2 * (N + 1) * NS + N * NU;
    return gains > stage ? gains : stage;
}

// Dynamic LDS floats of the trajectory kernel for padded sizes NS, NU
// (reverse mode adds the w trajectory).
__host__ __device__ inline int traj_dyn_floats(int N, int NS, int NU, int nc, bool adj)
{
    return N * nc + N * NS + traj_gain_floats(N, NS, NU) + N * NU + N * NS + (adj ? (N + 1) * NS : 0);
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

// Riccati sweep and rollout for 4 states and 2 inputs, held in the registers
// of one wave: lane (i, j) = 4 i + j of each row of 16 lanes owns entry
// (i, j) of the 4 x 4 blocks (rows 1-3 of the wave repeat row 0). Row i of a
// block reaches lane (i, j) by quad broadcasts, column j by rotations of the
// row by 4, 8 and 12 lanes, so the sweep needs no barrier. Per step, with P = P_{t+1}:
//   (a) PA = P A, PAT = (P A)^T (P symmetric), PB_{i, j mod 2} = (P B), w = P f_t + p;
//   (b) Qxx = H_t + A^T PA and its transpose, Qux_{i mod 2, j} = (B^T PA),
//       Qux^T, Quu = 2Q_u + B^T PB, qu = r_t + B^T w, qx = h_t + A^T w;
//   (c) K = -Quu^{-1} Qux, k = -Quu^{-1} qu (2 x 2 inverse by its adjugate),
//       P_t = Qxx - Qux^T Quu^{-1} Qux averaged with its transpose,
//       p_t = qx - Qux^T Quu^{-1} qu.
// The sums over rows run in the lane's rotation order, so lanes that hold
// the same entry may differ in the last bits; P_t is made exactly symmetric
// by one ds_bpermute per step. The step-dependent LDS terms
// of step t - 1 are read while step t computes. Gains go to Kall[t][2][5];
// the rollout then keeps dx_r in lane r (quads repeat) and writes dx
// (forward: dX[t][4], du in dU[t][2]; reverse: w in W[t + 1][4]).
template <bool ADJ>
__device__ __forceinline__ void riccati_regs_42(const float* A, const float* B, const float* Q2, const float* R2,
                                                const int* hmap, const int* gmap, const float* Hq, const float* qr,
                                                const float* rin, const float* off, float* Kall, float* dX, float* dU,
                                                float* W, int N, int nc, float x0dev)
{
    const int lane = threadIdx.x & 15;
    const int i = lane >> 2, j = lane & 3, a = i & 1, b = j & 1;
    int km[4];
    km[0] = i;
    km[1] = row_ror_i<4>(i);
    km[2] = row_ror_i<8>(i);
    km[3] = row_ror_i<12>(i);
    float Acol[4], Bcol[4], Arot[4], Brot[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Acol[k] = A[k * 4 + j];
        Bcol[k] = B[k * 2 + b];
        Arot[k] = A[km[k] * 4 + i];
        Brot[k] = B[km[k] * 2 + a];
    }
    const float q2ij = Q2[i * 4 + j], q2ji = Q2[j * 4 + i], r2ab = R2[a * 2 + b];
    const int hmij = hmap[i * 4 + j], hmji = hmap[j * 4 + i], gmi = ADJ ? -1 : gmap[i];
    const int tsrc = (((int)threadIdx.x & ~15) | (i <= j ? lane : j * 4 + i)) << 2;   // ds_bpermute byte address
    float Pv = q2ij + (hmij >= 0 ? Hq[(N - 1) * nc + hmij] : 0.f);
    float pv = qr[(N - 1) * 4 + i] + (gmi >= 0 ? Hq[(N - 1) * nc + gmi] : 0.f);
    // step-dependent terms of step t: H_{t-1} (i, j) and (j, i), h_{t-1}(i), f_t, r_t
    float nHij = 0.f, nHji = 0.f, nh = 0.f, nf[4], nr;
    auto fetch = [&](int t) {
        if (t >= 1) {
            const float* hq = Hq + (t - 1) * nc;
            nHij = q2ij + (hmij >= 0 ? hq[hmij] : 0.f);
            nHji = q2ji + (hmji >= 0 ? hq[hmji] : 0.f);
            nh = qr[(t - 1) * 4 + i] + (gmi >= 0 ? hq[gmi] : 0.f);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) nf[k] = off[t * 4 + k];
        nr = rin[t * 2 + a];
    };
    fetch(N - 1);
    for (int t = N - 1; t >= 0; --t) {
        const float Hij = nHij, Hji = nHji, h = nh, r = nr;
        float f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = nf[k];
        if (t >= 1) fetch(t - 1);
        // (a)
        const float Pb[4] = {quad_bcast<0>(Pv), quad_bcast<1>(Pv), quad_bcast<2>(Pv), quad_bcast<3>(Pv)};
        const float Pr[4] = {Pv, row_ror<4>(Pv), row_ror<8>(Pv), row_ror<12>(Pv)};
        float PA = 0.f, PAT = 0.f, PB = 0.f, w = pv;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            PA += Pb[k] * Acol[k];
            PB += Pb[k] * Bcol[k];
            w += Pb[k] * f[k];
            PAT += Pr[k] * Arot[k];
        }
        // (b)
        const float PAr[4] = {PA, row_ror<4>(PA), row_ror<8>(PA), row_ror<12>(PA)};
        const float PBr[4] = {PB, row_ror<4>(PB), row_ror<8>(PB), row_ror<12>(PB)};
        const float wr[4] = {w, row_ror<4>(w), row_ror<8>(w), row_ror<12>(w)};
        float Qux = 0.f, Quu = r2ab, qu = r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Qux += Brot[k] * PAr[k];
            Quu += Brot[k] * PBr[k];
            qu += Brot[k] * wr[k];
        }
        // (c) Quu entries from the lanes of the other row / column parity
        const float xo = dpp_xor1(Quu);
        const float y = row_ror<4>(Quu), yo = row_ror<4>(xo);
        const float Q00 = a ? (b ? yo : y) : (b ? xo : Quu);
        const float Q11 = a ? (b ? Quu : xo) : (b ? y : yo);
        const float Q01 = a ? (b ? y : yo) : (b ? Quu : xo);
        const float idet = __builtin_amdgcn_rcpf(Q00 * Q11 - Q01 * Q01);
        const float I00 = Q11 * idet, I11 = Q00 * idet, I01 = -Q01 * idet;
        const float uxr = row_ror<4>(Qux);
        const float U0j = a ? uxr : Qux, U1j = a ? Qux : uxr;
        const float G0j = I00 * U0j + I01 * U1j, G1j = I01 * U0j + I11 * U1j;
        const float qur = row_ror<4>(qu);
        const float qu0 = a ? qur : qu, qu1 = a ? qu : qur;
        const float g0 = I00 * qu0 + I01 * qu1, g1 = I01 * qu0 + I11 * qu1;
        float* Kt = Kall + t * 10;
        if (threadIdx.x < 4) {
            Kt[j] = -G0j;
            Kt[5 + j] = -G1j;
            if (j == 0) {
                Kt[4] = -g0;
                Kt[9] = -g1;
            }
        }
        if (t >= 1) {
            float Qxx = Hij, qx = h, QxxT = Hji, QuxT = 0.f;
            const float PATb[4] = {quad_bcast<0>(PAT), quad_bcast<1>(PAT), quad_bcast<2>(PAT), quad_bcast<3>(PAT)};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Qxx += Arot[k] * PAr[k];
                qx += Arot[k] * wr[k];
                QxxT += Acol[k] * PATb[k];
                QuxT += Bcol[k] * PATb[k];
            }
            const float U0i = quad_bcast<0>(QuxT), U1i = quad_bcast<1>(QuxT);
            const float G0i = I00 * U0i + I01 * U1i, G1i = I01 * U0i + I11 * U1i;
            const float pij = Qxx - (U0i * G0j + U1i * G1j);
            const float pji = QxxT - (U0j * G0i + U1j * G1i);
            // exact symmetry: lane (i, j), i > j, takes the value of lane (j, i)
            // (an antisymmetric part would not be removed by the averaging
            // and grows along the sweep)
            Pv = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(
                     tsrc, __builtin_bit_cast(int, 0.5f * (pij + pji))));
            pv = qx - (U0i * g0 + U1i * g1);
        }
    }
    // rollout: lane r = j of each quad holds dx_r
    float Ar[4], Br[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) Ar[k] = A[j * 4 + k];
    Br[0] = B[j * 2];
    Br[1] = B[j * 2 + 1];
    float xv = x0dev;
    float nK[10], nft;
    auto fetchK = [&](int t) {
#pragma unroll
        for (int q = 0; q < 10; ++q) nK[q] = Kall[t * 10 + q];
        nft = off[t * 4 + j];
    };
    fetchK(0);
    for (int t = 0; t < N; ++t) {
        float K[10];
#pragma unroll
        for (int q = 0; q < 10; ++q) K[q] = nK[q];
        const float ft = nft;
        if (t + 1 < N) fetchK(t + 1);
        const float xb[4] = {quad_bcast<0>(xv), quad_bcast<1>(xv), quad_bcast<2>(xv), quad_bcast<3>(xv)};
        float u0 = K[4], u1 = K[9], xn = ft;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            u0 += K[k] * xb[k];
            u1 += K[5 + k] * xb[k];
            xn += Ar[k] * xb[k];
        }
        xn += Br[0] * u0 + Br[1] * u1;
        if (threadIdx.x < 4) {
            if (ADJ) W[(t + 1) * 4 + j] = xn;
            else dX[t * 4 + j] = xn;
            if (!ADJ && j < 2) dU[t * 2 + j] = j == 0 ? u0 : u1;
        }
        xv = xn;
    }
}

// Trajectory QP of one scenario per workgroup. State/input sizes are padded
// to the compile-time NS >= n_s, NU >= n_u with zero dynamics rows/columns
// and an identity input-cost block, so every small product unrolls.
template <int NS, int NU, bool ADJ>
__global__ void __launch_bounds__(traj_threads(NS, NU)) traj_phase_kernel(DevProblem P, int obstacle_free,
                                                                          float* hq_save, TrajAdjoint TA)
{
    constexpr int TT = traj_threads(NS, NU);
    constexpr int NSU = NS + 1;
    __shared__ float A[NS * NS], B[NS * NU], Q2[NS * NS], R2[NU * NU], cdyn[NS];
    __shared__ int hmap[NS * NS], gmap[NS], pmap[NS];
    __shared__ float Pm[NS * NS], pv[NS], PA[NS * NS], PB[NS * NU], wv[NS];
    __shared__ float Quu[NU * NU], Qux[NU * NS], qu[NU], Qxx[NS * NS], qx[NS];
    __shared__ float xbuf[2][NS];
    extern __shared__ float dyn[];
    const int s = blockIdx.x;
    if (!ADJ && !obstacle_free && P.done[s]) return;
    const int tid = threadIdx.x;
    const int ns = P.n_s, nu = P.n_u, N = P.N, nq = P.nq, nc = P.nc;
    // deviation coordinates about the current iterate (else base point 0)
    const bool dev = !ADJ && !obstacle_free;
    float* Hq = dyn;                       // [N][nc] reduced contributions
    float* qr = Hq + N * nc;               // [N][NS] stage gradients g_t (reverse: -xbar_t), t = 1..N
    float* Kall = qr + N * NS;             // [N][NU][NS+1] gains [K | k]
    float* sx = Kall;                      // staged before the sweep: [N+1][NS] x (reverse: x^K)
    float* sxr = sx + (N + 1) * NS;        //   [N+1][NS] x_ref
    float* su = sxr + (N + 1) * NS;        //   [N][NU] u (reverse: u^K)
    float* rin = Kall + traj_gain_floats(N, NS, NU);   // [N][NU] input gradients 2 Q_u u^k_t (reverse: -ubar_t)
    float* off = rin + N * NU;             // [N][NS] dynamics offsets f_t (c when the base is 0)
    float* wl = off + N * NS;              // reverse: [N+1][NS] w_t

    // 0. padded model and cost, pose-coordinate maps
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
        B[e] = (i < ns && j < nu) ? P.B_dyn[i * nu + j] : 0.f;
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
        // four steps per thread: the pose partials are summed as float4
        const int N4 = (N + 3) / 4;
        for (int e = tid; e < N4 * NS; e += TT) {
            const int t4 = e / NS, i = e % NS;
            const int a = pmap[i];
            float4 part = make_float4(0.f, 0.f, 0.f, 0.f);
            if (TA.qpart && a >= 0)
                part = strided_sum4(reinterpret_cast<const float4*>(TA.qpart + (size_t)a * 64) + t4, (size_t)nq * 16,
                                    wr.x, wr.y);
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
        if (!obstacle_free) {
            // four steps per thread, the partials summed as float4
            const int N4 = (N + 3) / 4;
            for (int e = tid; e < N4 * nc; e += TT) {
                const int cc = e / N4, t4 = e % N4;
                const float4 v = strided_sum4(reinterpret_cast<const float4*>(P.contrib + (size_t)cc * 64) + t4,
                                              (size_t)nc * 16, wr.x, wr.y);
                const float vq[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = 4 * t4 + q;
                    if (t >= N) break;
                    Hq[t * nc + cc] = vq[q];
                    if (hq_save) hq_save[((size_t)s * N + t) * nc + cc] = vq[q];
                }
            }
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
        for (int e = tid; e < N * NS; e += TT) {
            const int t = e / NS, i = e % NS;
            double acc = (double)cdyn[i];
            if (dev) {
                acc -= (double)sx[(t + 1) * NS + i];
#pragma unroll
                for (int j = 0; j < NS; ++j) acc += (double)A[i * NS + j] * (double)sx[t * NS + j];
#pragma unroll
                for (int j = 0; j < NU; ++j) acc += (double)B[i * NU + j] * (double)su[t * NU + j];
            }
            off[e] = (float)acc;
        }
    }
    __syncthreads();
    float* xo = P.x + (size_t)s * (N + 1) * ns;
    float* uo = P.u + (size_t)s * N * nu;
    float* dX = ADJ ? wl : qr;             // forward: dx_t at (t-1) * NS, t = 1..N; reverse: w_t at t * NS
    float* dU = rin;                       // forward: du_t at t * NU
    if constexpr (NS == 4 && NU == 2) {
        // 2-3. the sweep and the rollout in the registers of wave 0
        if (tid < 64) {
            const int r = tid & 3;
            float x0d = 0.f;
            if (!ADJ && r < ns) {
                const float x0v = P.x0[(size_t)s * ns + r];
                x0d = dev ? x0v - xo[r] : x0v;
            }
            if (ADJ && tid < 4) wl[tid] = 0.f;
            riccati_regs_42<ADJ>(A, B, Q2, R2, hmap, gmap, Hq, qr, rin, off, Kall, dX, dU, wl, N, nc, x0d);
        }
        __syncthreads();
    } else {
    // 2. backward Riccati sweep, V_t(x) = 1/2 x^T P x + p^T x, P_N = H_N.
    //    Every phase is one strided dot product per thread, so a wave never
    //    runs several output types one after the other:
    //      out = bias + sum_k X[k * xs] Y[k * ys]
    //    (a) PA = P A, PB = P B, w = P f_t + p;
    //    (b) Quu = 2Q_u + B^T PB, Qux = B^T PA, qu = B^T w + input gradient,
    //        Qxx = H_t + A^T PA, qx = h_t + A^T w (t >= 1);
    //    (c) gains [K | k] = -Quu^{-1} [Qux | qu] and the update
    //        P_t = Qxx + Qux^T K (symmetrised), p_t = qx + Qux^T k: each
    //        thread factors the small Quu itself, so (c) needs no extra barrier.
    //    (Folding (a) into (b) for tiny NS, NS^2 terms per output, measured
    //    slower than the extra barrier on gfx950.)
    constexpr bool kFold = false;
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
    __syncthreads();
    for (int t = N - 1; t >= 0; --t) {
        const float* ft = off + t * NS;
        float bias = b_q2;
        if (b_type == 2) bias = rin[t * NU + b_i];
        else if (b_type == 3 && t >= 1) bias += b_hm >= 0 ? Hq[(t - 1) * nc + b_hm] : 0.f;
        else if (b_type == 4 && t >= 1) bias = qr[(t - 1) * NS + b_i] + (b_hm >= 0 ? Hq[(t - 1) * nc + b_hm] : 0.f);
        if (!kFold) {
            // (a)
            if (a_type >= 0) {
                const float* X = Pm + a_i * NS;
                const float* Y = a_type == 0 ? A + a_j : (a_type == 1 ? B + a_j : ft);
                const int ys = a_type == 0 ? NS : (a_type == 1 ? NU : 1);
                float acc = a_type == 2 ? pv[a_i] : 0.f;
#pragma unroll
                for (int k2 = 0; k2 < NS; ++k2) acc += X[k2] * Y[k2 * ys];
                float* O = a_type == 0 ? PA + a_i * NS + a_j : (a_type == 1 ? PB + a_i * NU + a_j : wv + a_i);
                *O = acc;
            }
            __syncthreads();
        }
        // (b)
        if (b_type >= 0 && (t >= 1 || b_type <= 2)) {
            // X: column b_i of B (types 0-2) or of A (types 3-4)
            const float* X = b_type <= 2 ? B + b_i : A + b_i;
            const int xs = b_type <= 2 ? NU : NS;
            float acc = bias;
            if (kFold) {
                // Y column j of P B, P A or the vector P f_t + p, formed here
#pragma unroll
                for (int k2 = 0; k2 < NS; ++k2) {
                    float y;
                    if (b_type == 0) {
                        y = 0.f;
#pragma unroll
                        for (int l = 0; l < NS; ++l) y += Pm[k2 * NS + l] * B[l * NU + b_j];
                    } else if (b_type == 1 || b_type == 3) {
                        y = 0.f;
#pragma unroll
                        for (int l = 0; l < NS; ++l) y += Pm[k2 * NS + l] * A[l * NS + b_j];
                    } else {
                        y = pv[k2];
#pragma unroll
                        for (int l = 0; l < NS; ++l) y += Pm[k2 * NS + l] * ft[l];
                    }
                    acc += X[k2 * xs] * y;
                }
            } else {
                const float* Y = b_type == 0 ? PB + b_j : ((b_type == 1 || b_type == 3) ? PA + b_j : wv);
                const int ys = b_type == 0 ? NU : ((b_type == 1 || b_type == 3) ? NS : 1);
#pragma unroll
                for (int k2 = 0; k2 < NS; ++k2) acc += X[k2 * xs] * Y[k2 * ys];
            }
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
        __syncthreads();
    }
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
            for (int j = 0; j < NS; ++j) acc += A[j * NS + tid] * (xbuf[cur][j] + qr[t * NS + j]);
            xbuf[cur ^ 1][tid] = acc;
        }
        cur ^= 1;
        __syncthreads();
    }
    if (tid < ns) TA.gx0[(size_t)s * ns + tid] += (double)xbuf[cur][tid];
}

// ------------------------------------------------------------------------
// scale LP (Sec. III-A eq. scale_opt) through its dual (Sec. III-B eq.
// scale_opt_dual) in standard form
//   min dp^T mu  s.t.  b^T lam = 1,  A^T lam + Cp^T mu = 0,  lam, mu >= 0,
// by a two-phase revised simplex (Bland's rule) with an explicit
// (dim+1) x (dim+1) basis inverse in registers; columns are produced on the
// fly from the geometry. The optimal basis is re-solved directly at the end.
// ------------------------------------------------------------------------

template <int DIM, class Cols>
__device__ int revised_simplex(const Cols& cols, float& alpha, float* xB_out, int* basis_out)
{
    constexpr int m = DIM + 1;
    const int n = cols.n();
    float Bi[m * m];
    float xB[m];
    int basis[m];
#pragma unroll
    for (int i = 0; i < m; ++i) {
#pragma unroll
        for (int j = 0; j < m; ++j) Bi[i * m + j] = i == j ? 1.f : 0.f;
        xB[i] = i == 0 ? 1.f : 0.f;
        basis[i] = n + i;
    }
    const float ctol = 1e-6f * (1.f + cols.cmax());
    const float ptol = 1e-6f;
    int status = 0;
    for (int phase = 1; phase <= 2 && status == 0; ++phase) {
        int it = 0;
        for (; it < 64; ++it) {
            float cB[m];
#pragma unroll
            for (int i = 0; i < m; ++i)
                cB[i] = phase == 1 ? (basis[i] >= n ? 1.f : 0.f) : (basis[i] < n ? cols.cost(basis[i]) : 0.f);
            float pi[m];
#pragma unroll
            for (int q = 0; q < m; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int i = 0; i < m; ++i) acc += cB[i] * Bi[i * m + q];
                pi[q] = acc;
            }
            int enter = -1;
            float Eq[m];
            for (int j = 0; j < n && enter < 0; ++j) {
                bool basic = false;
#pragma unroll
                for (int i = 0; i < m; ++i) basic |= basis[i] == j;
                if (basic) continue;
                float E[m];
                cols.col(j, E);
                float rc = phase == 1 ? 0.f : cols.cost(j);
#pragma unroll
                for (int q = 0; q < m; ++q) rc -= pi[q] * E[q];
                if (rc < -ctol) {
                    enter = j;
#pragma unroll
                    for (int q = 0; q < m; ++q) Eq[q] = E[q];
                }
            }
            if (enter < 0) break;
            float u[m];
#pragma unroll
            for (int i = 0; i < m; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int q = 0; q < m; ++q) acc += Bi[i * m + q] * Eq[q];
                u[i] = acc;
            }
            int leave = -1;
            float best = 0.f;
#pragma unroll
            for (int i = 0; i < m; ++i) {
                if (u[i] > ptol) {
                    const float ratio = xB[i] / u[i];
                    if (leave < 0 || ratio < best || (ratio == best && basis[i] < basis[leave])) {
                        leave = i;
                        best = ratio;
                    }
                }
            }
            if (leave < 0) { status = 2; break; }
            float ur = 0.f;
#pragma unroll
            for (int i = 0; i < m; ++i) ur = i == leave ? u[i] : ur;
            const float iu = 1.f / ur;
            float rowB[m], xr = 0.f;
#pragma unroll
            for (int q = 0; q < m; ++q) {
                float v = 0.f;
#pragma unroll
                for (int i = 0; i < m; ++i) v = i == leave ? Bi[i * m + q] : v;
                rowB[q] = v * iu;
            }
#pragma unroll
            for (int i = 0; i < m; ++i) xr = i == leave ? xB[i] : xr;
            xr *= iu;
#pragma unroll
            for (int i = 0; i < m; ++i) {
                if (i == leave) {
#pragma unroll
                    for (int q = 0; q < m; ++q) Bi[i * m + q] = rowB[q];
                    xB[i] = xr;
                    basis[i] = enter;
                } else {
#pragma unroll
                    for (int q = 0; q < m; ++q) Bi[i * m + q] -= u[i] * rowB[q];
                    xB[i] = fmaxf(0.f, xB[i] - u[i] * xr);
                }
            }
        }
        if (it >= 64) status = 3;
        if (phase == 1 && status == 0) {
            // pivot zero-level artificials out of the basis
#pragma unroll
            for (int i = 0; i < m; ++i) {
                if (basis[i] < n) continue;
                int piv = -1;
                float bestv = 1e-5f, uu[m];
                for (int j = 0; j < n; ++j) {
                    bool basic = false;
#pragma unroll
                    for (int k = 0; k < m; ++k) basic |= basis[k] == j;
                    if (basic) continue;
                    float E[m];
                    cols.col(j, E);
                    float ui = 0.f;
#pragma unroll
                    for (int q = 0; q < m; ++q) ui += Bi[i * m + q] * E[q];
                    if (fabsf(ui) > bestv) {
                        bestv = fabsf(ui);
                        piv = j;
#pragma unroll
                        for (int k = 0; k < m; ++k) {
                            float acc = 0.f;
#pragma unroll
                            for (int q = 0; q < m; ++q) acc += Bi[k * m + q] * E[q];
                            uu[k] = acc;
                        }
                    }
                }
                if (piv < 0) continue;
                const float iu = 1.f / uu[i];
                float rowB[m];
#pragma unroll
                for (int q = 0; q < m; ++q) rowB[q] = Bi[i * m + q] * iu;
                const float xr = xB[i] * iu;
#pragma unroll
                for (int k = 0; k < m; ++k) {
                    if (k == i) {
#pragma unroll
                        for (int q = 0; q < m; ++q) Bi[k * m + q] = rowB[q];
                        xB[k] = xr;
                    } else {
#pragma unroll
                        for (int q = 0; q < m; ++q) Bi[k * m + q] -= uu[k] * rowB[q];
                        xB[k] -= uu[k] * xr;
                    }
                }
                basis[i] = piv;
            }
        }
    }
    // re-solve the optimal basis directly: Bmat x_B = f, pi^T Bmat = c_B^T
    float Bm[m * m];
#pragma unroll
    for (int i = 0; i < m; ++i) {
        float E[m];
        if (basis[i] < n) cols.col(basis[i], E);
        else {
#pragma unroll
            for (int q = 0; q < m; ++q) E[q] = q == basis[i] - n ? 1.f : 0.f;
        }
#pragma unroll
        for (int q = 0; q < m; ++q) Bm[q * m + i] = E[q];   // column i of the basis matrix
    }
    // Gauss-Jordan inverse with partial pivoting
    float Inv[m * m];
#pragma unroll
    for (int i = 0; i < m; ++i)
#pragma unroll
        for (int j = 0; j < m; ++j) Inv[i * m + j] = i == j ? 1.f : 0.f;
#pragma unroll
    for (int k = 0; k < m; ++k) {
        int p = k;
        float bv = fabsf(Bm[k * m + k]);
#pragma unroll
        for (int i = k + 1; i < m; ++i)
            if (fabsf(Bm[i * m + k]) > bv) { bv = fabsf(Bm[i * m + k]); p = i; }
        if (bv > 0.f) {
#pragma unroll
            for (int i = k + 1; i < m; ++i) {
                if (i == p) {
#pragma unroll
                    for (int j = 0; j < m; ++j) {
                        float t1 = Bm[k * m + j]; Bm[k * m + j] = Bm[i * m + j]; Bm[i * m + j] = t1;
                        float t2 = Inv[k * m + j]; Inv[k * m + j] = Inv[i * m + j]; Inv[i * m + j] = t2;
                    }
                }
            }
            const float ip = 1.f / Bm[k * m + k];
#pragma unroll
            for (int j = 0; j < m; ++j) { Bm[k * m + j] *= ip; Inv[k * m + j] *= ip; }
#pragma unroll
            for (int i = 0; i < m; ++i) {
                if (i == k) continue;
                const float f = Bm[i * m + k];
#pragma unroll
                for (int j = 0; j < m; ++j) { Bm[i * m + j] -= f * Bm[k * m + j]; Inv[i * m + j] -= f * Inv[k * m + j]; }
            }
        } else {
            status = status ? status : 4;
        }
    }
    float cB[m];
#pragma unroll
    for (int i = 0; i < m; ++i) cB[i] = basis[i] < n ? cols.cost(basis[i]) : 0.f;
    float pi0 = 0.f;
#pragma unroll
    for (int i = 0; i < m; ++i) pi0 += cB[i] * Inv[i * m + 0];
#pragma unroll
    for (int i = 0; i < m; ++i) {
        xB_out[i] = fmaxf(0.f, Inv[i * m + 0]);   // f = e_0
        basis_out[i] = basis[i];
    }
    alpha = -pi0;
    return status;
}

// columns of the ADMM problem's pair (part frame through the pose)
template <int DIM>
struct PairCols {
    int nr, no, fo0;
    const float4* rf;
    const float4* of;
    const double* d64;
    float R[DIM * DIM];
    double pos64[DIM];
    float cmx;
    __device__ int n() const { return nr + no; }
    __device__ float cmax() const { return cmx; }
    __device__ float cost(int j) const {
        if (j < nr) return 0.f;
        return face_offset(d64, fo0 + j - nr, of[j - nr], pos64, DIM);
    }
    __device__ void col(int j, float (&E)[DIM + 1]) const {
        if (j < nr) {
            const float4 f = rf[j];
            E[0] = f.w;
            E[1] = f.x;
            E[2] = f.y;
            if (DIM == 3) E[DIM] = f.z;
        } else {
            const float4 f = of[j - nr];
            const float c[3] = {f.x, f.y, f.z};
            E[0] = 0.f;
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int r = 0; r < DIM; ++r) acc += R[r * DIM + q] * c[r];
                E[1 + q] = acc;
            }
        }
    }
};

// initial dual iterate from the scale LP at the current trajectory:
// y = (lam*, mu*, max(alpha* - 1, 0)); optionally alpha* per pair.
template <int DIM>
__global__ void __launch_bounds__(256) init_pairs_kernel(DevProblem P, float* alpha_out, int write_y)
{
    const int b = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int N = P.N, t = lane + 1;
    if (b >= P.n_blocks || t > N) return;
    const int4 blk = P.blocks[b];
    const int s = blk.x, part = uniform(blk.y), obs = uniform(blk.z);
    const int fr0 = uniform(P.part_face_ptr[part]);
    const int fo0 = uniform(P.obs_face_ptr[obs]);
    PairCols<DIM> pc;
    pc.nr = uniform(P.part_face_ptr[part + 1] - fr0);
    pc.no = uniform(P.obs_face_ptr[obs + 1] - fo0);
    pc.rf = P.part_faces + fr0;
    pc.of = P.obs_faces + fo0;
    Pose<DIM> ps;
    make_pose<DIM>(P, P.x + ((size_t)s * (N + 1) + t) * P.n_s, part, ps);
#pragma unroll
    for (int i = 0; i < DIM * DIM; ++i) pc.R[i] = ps.R[i];
#pragma unroll
    for (int i = 0; i < DIM; ++i) pc.pos64[i] = ps.pos64[i];
    pc.fo0 = fo0;
    pc.d64 = P.obs_d64;
    float cm = 0.f;
    for (int l = 0; l < pc.no; ++l) cm = fmaxf(cm, fabsf(pc.cost(pc.nr + l)));
    pc.cmx = cm;
    float alpha, xB[DIM + 1];
    int basis[DIM + 1];
    revised_simplex<DIM>(pc, alpha, xB, basis);
    if (alpha_out) alpha_out[(size_t)b * N + t - 1] = alpha;
    if (write_y) {
        float* yb = P.y + P.block_yoff[b] + (t - 1);
        const int nrow = pc.nr + pc.no;
        for (int j = 0; j < nrow; ++j) {
            float v = 0.f;
#pragma unroll
            for (int i = 0; i <= DIM; ++i) v = basis[i] == j ? xB[i] : v;
            yb[j * N] = v;
        }
        yb[nrow * N] = fmaxf(alpha - 1.f, 0.f);
    }
}

// ------------------------------------------------------------------------
// stateless batch entry points
// ------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(256) pair_qp_batch_kernel(int n_pairs, const int* row_ptr, const float* K,
                                                            const float* kappa, const float* yhat,
                                                            const float* bhat, float eps, int max_sweeps,
                                                            float* y, float* r, int* status)
{
    constexpr int NV = DIM + 2;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    const int r0 = row_ptr[p], n = row_ptr[p + 1] - r0;
    GenRows<DIM> gr;
    gr.n = n;
    gr.K = K + (size_t)r0 * (DIM + 1);
    gr.kap = kappa + r0;
    gr.yh = yhat + r0;
    gr.eps = eps;
#pragma unroll
    for (int c = 0; c <= DIM; ++c) gr.bh[c] = bhat[(size_t)p * (DIM + 1) + c];
    // warm start v = K^T yhat + bhat; nu makes the largest kappa-row stationary
    float z[NV];
#pragma unroll
    for (int c = 0; c <= DIM; ++c) z[c] = gr.bh[c];
    for (int l = 0; l < n; ++l)
#pragma unroll
        for (int c = 0; c <= DIM; ++c) z[c] += gr.yh[l] * gr.K[l * (DIM + 1) + c];
    float best = -1.f, nu = 0.f;
    for (int l = 0; l < n; ++l) {
        if (gr.kap[l] > 0.f && gr.yh[l] > best) {
            best = gr.yh[l];
            float s = 0.f;
#pragma unroll
            for (int c = 0; c <= DIM; ++c) s += gr.K[l * (DIM + 1) + c] * z[c];
            nu = s / gr.kap[l];
        }
    }
    z[DIM + 1] = nu;
    const int sw = dual_newton<NV>(gr, z, max_sweeps);
    float rr[DIM + 1];
#pragma unroll
    for (int c = 0; c <= DIM; ++c) rr[c] = gr.bh[c];
    for (int l = 0; l < n; ++l) {
        float D = 0.f, s = -gr.kap[l] * z[DIM + 1];
#pragma unroll
        for (int c = 0; c <= DIM; ++c) {
            const float k = gr.K[l * (DIM + 1) + c];
            D += k * k;
            s += k * z[c];
        }
        const float yl = fmaxf(0.f, gr.yh[l] - s / (eps * D));
        y[r0 + l] = yl;
#pragma unroll
        for (int c = 0; c <= DIM; ++c) rr[c] += yl * gr.K[l * (DIM + 1) + c];
    }
#pragma unroll
    for (int c = 0; c <= DIM; ++c) r[(size_t)p * (DIM + 1) + c] = rr[c];
    status[p] = sw;
}

template <int DIM>
struct MemCols {
    int nr, no;
    const float* A;
    const float* b;
    const float* Cp;
    const float* dp;
    float cmx;
    __device__ int n() const { return nr + no; }
    __device__ float cmax() const { return cmx; }
    __device__ float cost(int j) const { return j < nr ? 0.f : dp[j - nr]; }
    __device__ void col(int j, float (&E)[DIM + 1]) const {
        if (j < nr) {
            E[0] = b[j];
#pragma unroll
            for (int q = 0; q < DIM; ++q) E[1 + q] = A[j * DIM + q];
        } else {
            E[0] = 0.f;
#pragma unroll
            for (int q = 0; q < DIM; ++q) E[1 + q] = Cp[(j - nr) * DIM + q];
        }
    }
};

template <int DIM>
__global__ void __launch_bounds__(256) scale_batch_kernel(int n_pairs, const int* a_ptr, const float* A,
                                                          const float* b, const int* o_ptr, const float* Cp,
                                                          const float* dp, float* alpha, float* lam,
                                                          float* mu, int* status)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    const int a0 = a_ptr[p], o0 = o_ptr[p];
    MemCols<DIM> mc;
    mc.nr = a_ptr[p + 1] - a0;
    mc.no = o_ptr[p + 1] - o0;
    mc.A = A + (size_t)a0 * DIM;
    mc.b = b + a0;
    mc.Cp = Cp + (size_t)o0 * DIM;
    mc.dp = dp + o0;
    float cm = 0.f;
    for (int l = 0; l < mc.no; ++l) cm = fmaxf(cm, fabsf(mc.dp[l]));
    mc.cmx = cm;
    float al, xB[DIM + 1];
    int basis[DIM + 1];
    const int st = revised_simplex<DIM>(mc, al, xB, basis);
    alpha[p] = al;
    for (int j = 0; j < mc.nr + mc.no; ++j) {
        float v = 0.f;
#pragma unroll
        for (int i = 0; i <= DIM; ++i) v = basis[i] == j ? xB[i] : v;
        if (j < mc.nr) lam[a0 + j] = v;
        else mu[o0 + j - mc.nr] = v;
    }
    status[p] = st;
}

// ------------------------------------------------------------------------
// misc kernels
// ------------------------------------------------------------------------

__global__ void fill_kernel(float* p, long long n, float v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void set_face_offsets_kernel(float4* faces, const double* d64, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) faces[i].w = (float)d64[i];
}

__global__ void fill_int_kernel(int* p, long long n, int v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// tracking cost F (Sec. IV-A eq. navigation_cost) of each scenario
__global__ void __launch_bounds__(64) cost_kernel(DevProblem P, float* out)
{
    const int s = blockIdx.x;
    const int ns = P.n_s, nu = P.n_u, N = P.N;
    float acc = 0.f;
    for (int e = threadIdx.x; e < N * (ns + nu); e += 64) {
        const int t = e / (ns + nu), k = e % (ns + nu);
        if (k < ns) {
            const float* xt = P.x + ((size_t)s * (N + 1) + t + 1) * ns;
            const float* xr = P.x_ref + ((size_t)s * (N + 1) + t + 1) * ns;
            float qa = 0.f;
            for (int j = 0; j < ns; ++j) qa += P.Q_s[k * ns + j] * (xt[j] - xr[j]);
            acc += (xt[k] - xr[k]) * qa;
        } else {
            const int i = k - ns;
            const float* ut = P.u + ((size_t)s * N + t) * nu;
            float qa = 0.f;
            for (int j = 0; j < nu; ++j) qa += P.Q_u[i * nu + j] * ut[j];
            acc += ut[i] * qa;
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x == 0) out[s] = acc;
}

__global__ void __launch_bounds__(64) min_alpha_kernel(DevProblem P, const float* alpha, float* out)
{
    const int s = blockIdx.x;
    const int2 r = P.scen_wg[s];
    float m = FLT_MAX;
    if (r.y > r.x) {
        const int b0 = P.wg_items[r.x].y, b1 = P.wg_items[r.y - 1].z;
        for (long long e = (long long)b0 * P.N + threadIdx.x; e < (long long)b1 * P.N; e += 64) m = fminf(m, alpha[e]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    if (threadIdx.x == 0) out[s] = m;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

struct Variant { int dim, mr, mo; };
static const Variant kVariants[] = {{2, 4, 16}, {2, 8, 32}, {3, 6, 24}, {3, 8, 32}};

bool pair_variant_supported(int dim, int mr, int mo)
{
    for (const auto& v : kVariants)
        if (v.dim == dim && mr <= v.mr && mo <= v.mo) return true;
    return false;
}

// first compiled variant whose face limits fit the problem
static int pick_variant(const DevProblem& P)
{
    for (int i = 0; i < 4; ++i)
        if (kVariants[i].dim == P.dim && P.max_part_faces <= kVariants[i].mr &&
            P.max_obs_faces <= kVariants[i].mo)
            return i;
    return -1;
}

template <int DIM, int MR, int MO>
static void launch_pair_g(const DevProblem& P, int W, int G, int grid, hipStream_t st)
{
    const int nc = P.nc;
    const int nw = pair_waves_per_block(P.N, G);
    const size_t lds = (size_t)W * (MR + MO) * sizeof(float4) + (size_t)W * nc * 64 * sizeof(float) +
                       2 * (size_t)W * nw * sizeof(float);
    dim3 blk(64 * W * nw), grd(grid);
    if (G == 4) hipLaunchKernelGGL((pair_phase_kernel<DIM, MR, MO, 4>), grd, blk, lds, st, P);
    else if (G == 2) hipLaunchKernelGGL((pair_phase_kernel<DIM, MR, MO, 2>), grd, blk, lds, st, P);
    else hipLaunchKernelGGL((pair_phase_kernel<DIM, MR, MO, 1>), grd, blk, lds, st, P);
}

bool pair_group_supported(int N, int W, int G)
{
    return (G == 1 || G == 2 || G == 4) && W >= 1 && W * pair_waves_per_block(N, G) <= 8;
}

hipError_t launch_pair_phase(const DevProblem& P, int W, int G, int grid, hipStream_t st)
{
    if (!pair_group_supported(P.N, W, G)) return hipErrorInvalidValue;
    switch (pick_variant(P)) {
    case 0: launch_pair_g<2, 4, 16>(P, W, G, grid, st); break;
    case 1: launch_pair_g<2, 8, 32>(P, W, G, grid, st); break;
    case 2: launch_pair_g<3, 6, 24>(P, W, G, grid, st); break;
    case 3: launch_pair_g<3, 8, 32>(P, W, G, grid, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mult_phase(const DevProblem& P, int W, int grid, hipStream_t st)
{
    const int v = pick_variant(P);
    const size_t lds = (size_t)W * sizeof(float);
    dim3 blk(64 * W), grd(grid);
    switch (v) {
    case 0: hipLaunchKernelGGL((mult_phase_kernel<2, 4, 16>), grd, blk, lds, st, P); break;
    case 1: hipLaunchKernelGGL((mult_phase_kernel<2, 8, 32>), grd, blk, lds, st, P); break;
    case 2: hipLaunchKernelGGL((mult_phase_kernel<3, 6, 24>), grd, blk, lds, st, P); break;
    case 3: hipLaunchKernelGGL((mult_phase_kernel<3, 8, 32>), grd, blk, lds, st, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool ADJ>
static hipError_t launch_traj(const DevProblem& P, int obstacle_free, float* hq_save, const TrajAdjoint& TA,
                              hipStream_t st)
{
    dim3 g(P.n_scen);
    if (P.n_s <= 4 && P.n_u <= 2) {
        const dim3 b(traj_threads(4, 2));
        hipLaunchKernelGGL((traj_phase_kernel<4, 2, ADJ>), g, b,
                           sizeof(float) * traj_dyn_floats(P.N, 4, 2, P.nc, ADJ), st, P, obstacle_free, hq_save, TA);
    } else if (P.n_s <= 12 && P.n_u <= 4) {
        const dim3 b(traj_threads(12, 4));
        hipLaunchKernelGGL((traj_phase_kernel<12, 4, ADJ>), g, b,
                           sizeof(float) * traj_dyn_floats(P.N, 12, 4, P.nc, ADJ), st, P, obstacle_free, hq_save, TA);
    } else {
        const dim3 b(traj_threads(16, 8));
        hipLaunchKernelGGL((traj_phase_kernel<16, 8, ADJ>), g, b,
                           sizeof(float) * traj_dyn_floats(P.N, 16, 8, P.nc, ADJ), st, P, obstacle_free, hq_save, TA);
    }
    return hipGetLastError();
}

hipError_t launch_traj_phase(const DevProblem& P, int obstacle_free, hipStream_t st, float* hq_save)
{
    return launch_traj<false>(P, obstacle_free, hq_save, TrajAdjoint{}, st);
}

hipError_t launch_traj_adjoint(const DevProblem& P, const TrajAdjoint& TA, hipStream_t st)
{
    return launch_traj<true>(P, 0, nullptr, TA, st);
}

hipError_t launch_residual(const DevProblem& P, hipStream_t st)
{
    hipLaunchKernelGGL(residual_kernel, dim3(P.n_scen), dim3(64), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_init_pairs(const DevProblem& P, float* alpha_out, int write_y, hipStream_t st)
{
    const int grid = (P.n_blocks + 3) / 4;
    if (grid == 0) return hipSuccess;
    if (P.dim == 2)
        hipLaunchKernelGGL(init_pairs_kernel<2>, dim3(grid), dim3(256), 0, st, P, alpha_out, write_y);
    else
        hipLaunchKernelGGL(init_pairs_kernel<3>, dim3(grid), dim3(256), 0, st, P, alpha_out, write_y);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, long long n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_set_face_offsets(float4* faces, const double* d64, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_face_offsets_kernel, dim3((n + 255) / 256), dim3(256), 0, st, faces, d64, n);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long long g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_cost(const DevProblem& P, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(cost_kernel, dim3(P.n_scen), dim3(64), 0, st, P, out);
    return hipGetLastError();
}

hipError_t launch_min_alpha(const DevProblem& P, const float* alpha, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(min_alpha_kernel, dim3(P.n_scen), dim3(64), 0, st, P, alpha, out);
    return hipGetLastError();
}

hipError_t launch_pair_qp_batch(int n_pairs, int dim, const int* row_ptr, const float* K, const float* kappa,
                                const float* yhat, const float* bhat, float eps, int max_sweeps, float* y,
                                float* r, int* status, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (n_pairs + 255) / 256;
    if (dim == 2)
        hipLaunchKernelGGL(pair_qp_batch_kernel<2>, dim3(grid), dim3(256), 0, st, n_pairs, row_ptr, K, kappa,
                           yhat, bhat, eps, max_sweeps, y, r, status);
    else
        hipLaunchKernelGGL(pair_qp_batch_kernel<3>, dim3(grid), dim3(256), 0, st, n_pairs, row_ptr, K, kappa,
                           yhat, bhat, eps, max_sweeps, y, r, status);
    return hipGetLastError();
}

hipError_t launch_scale_batch(int n_pairs, int dim, const int* a_ptr, const float* A, const float* b,
                              const int* o_ptr, const float* Cp, const float* dp, float* alpha, float* lam,
                              float* mu, int* status, hipStream_t st)
{
    if (n_pairs <= 0) return hipSuccess;
    const int grid = (n_pairs + 255) / 256;
    if (dim == 2)
        hipLaunchKernelGGL(scale_batch_kernel<2>, dim3(grid), dim3(256), 0, st, n_pairs, a_ptr, A, b, o_ptr, Cp,
                           dp, alpha, lam, mu, status);
    else
        hipLaunchKernelGGL(scale_batch_kernel<3>, dim3(grid), dim3(256), 0, st, n_pairs, a_ptr, A, b, o_ptr, Cp,
                           dp, alpha, lam, mu, status);
    return hipGetLastError();
}

}  // namespace cadmm
