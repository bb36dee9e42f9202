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
#include "cadmm_solvers.h"

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

    // Gradient g and scale sc at z; with HESS the generalised Hessian of the
    // rows with y > 0 at z, with UNION of the rows with y > 0 at z or at zu.
    template <bool HESS, bool UNION = false>
    __device__ __forceinline__ void pass(const float (&z)[NV], float (&g)[NV], float (&H)[NV * NV],
                                         float& sc, const float* zu = nullptr) const
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
        float wu[DIM] = {};   // R v_r at zu
        if (UNION) {
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = 0.f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) acc += R[r * DIM + c] * zu[1 + c];
                wu[r] = acc;
            }
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
                    bool on = y > 0.f;
                    if (UNION) {
                        float su = -f.w * zu[DIM + 1];
#pragma unroll
                        for (int r = 0; r < DIM; ++r) su += a[r] * zu[1 + r];
                        on = on || yhR[m] - su * ieR[m] > 0.f;
                    }
                    const float act = on ? ieR[m] : 0.f;
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
                    bool on = y > 0.f;
                    if (UNION) {
                        float su = ch[0] * zu[0];
#pragma unroll
                        for (int r = 0; r < DIM; ++r) su += ch[1 + r] * wu[r];
                        on = on || yhO[m] - su * ieO[m] > 0.f;
                    }
                    const float act = on ? ieO[m] : 0.f;
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
            const bool g_on = yg > 0.f || (UNION && yhG - zu[0] * ieG > 0.f);
            H[0] = Mf[0] + 1.f + (g_on ? ieG : 0.f);
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
    float4* dcs = faces + WB * (MR + MO);             // [WB][MO] rounding of the obstacle normals
    double* d64s = reinterpret_cast<double*>(dcs + WB * MO);   // [WB][MO] FP64 obstacle face offsets
    float* red = reinterpret_cast<float*>(d64s + WB * MO);     // [WB][NC][64] contributions by step
    float* red_rd = red + WB * NC * 64;               // [W]
    int* red_un = reinterpret_cast<int*>(red_rd + W);
    const float eps = P.eps_prox;

    for (int wg = blockIdx.x; wg < P.n_wg; wg += gridDim.x) {
        const int4 item = P.wg_items[wg];
        const int s = uniform(item.x);
        const int b = uniform(item.y + bslot);
        // what depends only on (s, b, t) is loaded beside the block's
        // descriptor and the done flag (an empty slot loads a valid pair's
        // values and ignores them): the state entries of the pose and the
        // multipliers
        const int bq = min(b, item.z - 1), tq = min(t, N);
        PoseInputs<DIM> pin;
        load_pose_state<DIM>(P, P.x + ((size_t)s * (N + 1) + tq) * P.n_s, pin);
        const float zeta = P.zeta[(size_t)bq * N + tq - 1];
        float xi[DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r) xi[r] = P.xi[((size_t)bq * DIM + r) * N + tq - 1];
        const int4 bd = b < item.z ? P.bdesc[b] : int4{0, 0, 0, 0};
        if (P.done[s]) continue;                 // uniform over the workgroup
        const int fr0 = uniform(bd.x), fo0 = uniform(bd.y), yoff = uniform(bd.z);
        const int nrb = uniform(bd.w & 0xff), nob = uniform((bd.w >> 8) & 0xff), part = uniform(bd.w >> 16);
        // then, beside the faces, the part offset and the rows' proximal
        // centres (unconditional loads from clamped rows, all in flight at once)
        load_pose_offset<DIM>(P, part, pin);
        const float* yb = P.y + yoff + (tq - 1);
        float yRl[Rows::RR], yOl[Rows::RO];
#pragma unroll
        for (int m = 0; m < Rows::RR; ++m) yRl[m] = yb[max(0, min(q + G * m, nrb - 1)) * N];
#pragma unroll
        for (int m = 0; m < Rows::RO; ++m) yOl[m] = yb[(nrb + max(0, min(q + G * m, nob - 1))) * N];
        const float yG = yb[(nrb + nob) * N];
        // the block's faces into its LDS slot: every solver pass reads them,
        // and from LDS they are cheap reads instead of HBM round trips
        float4* fl = faces + bslot * (MR + MO);
        if (b < item.z && chunk == 0) {
            if (lane < nrb) fl[lane] = P.part_faces[fr0 + lane];
            else if (lane >= MR && lane - MR < nob) {
                fl[lane] = P.obs_faces[fo0 + lane - MR];
                dcs[bslot * MO + lane - MR] = P.obs_dc[fo0 + lane - MR];
                d64s[bslot * MO + lane - MR] = P.obs_d64[fo0 + lane - MR];
            }
        }
        __syncthreads();
        float con[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) con[c] = 0.f;
        float rd = 0.f;
        int unc = 0;
        if (b < item.z && t <= N) {
            Rows pr;
            pr.q = q;
            pr.nr = nrb;
            pr.no = nob;
            pr.rf = fl;
            pr.of = fl + MR;
            Pose<DIM> ps;
            make_pose_v<DIM>(pin.xp, pin.xa, pin.o, ps);
#pragma unroll
            for (int i = 0; i < DIM * DIM; ++i) pr.R[i] = ps.R[i];
            pr.bh[0] = 1.f + zeta;
#pragma unroll
            for (int r = 0; r < DIM; ++r) pr.bh[1 + r] = xi[r];
            // warm start v = K^T yhat + bhat, nu from the largest lambda row
            float v0 = 0.f, Sc[DIM] = {}, vr[DIM] = {};
#pragma unroll
            for (int m = 0; m < Rows::RR; ++m) {
                const int k = q + G * m;
                if (k < pr.nr) {
                    const float4 f = pr.rf[k];
                    const float yk = yRl[m];
                    pr.yhR[m] = yk;
                    const float D = f.x * f.x + f.y * f.y + (DIM == 3 ? f.z * f.z : 0.f);
                    pr.ieR[m] = __builtin_amdgcn_rcpf(eps * D);
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
                    const float yl = yOl[m];
                    pr.yhO[m] = yl;
                    const float dp = face_offset(d64s + bslot * MO, l, f, dcs[bslot * MO + l], ps.pos64, ps.pos, DIM);
                    float cn = 0.f;
#pragma unroll
                    for (int r = 0; r < DIM; ++r) cn += c[r] * c[r];
                    const float D = dp * dp + cn;
                    pr.ieO[m] = __builtin_amdgcn_rcpf(eps * D);
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
            pr.yhG = yG;
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
            const int sweeps = dual_newton<NV>(pr, z, P.max_sweeps, 1e-7f);
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
                const float* o = pin.o;
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
        // only the N step slots are written: the trajectory kernel reads
        // slots t >= N (float4 loads over four steps) but never uses them
        float* out = P.contrib + (size_t)wg * NC * 64;
        for (int e = threadIdx.x; e < NC * 64; e += blockDim.x) {
            if ((e & 63) >= N) continue;
            float acc = 0.f;
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
    extern __shared__ __align__(16) float lds[];
    const int W = blockDim.x >> 6;
    const int wave = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int N = P.N;
    // each wave's block geometry in LDS (faces, then the obstacle faces'
    // FP64 offsets and normal roundings): one parallel load per workgroup
    // instead of a dependent global load per face and lane
    float4* faces = reinterpret_cast<float4*>(lds) + wave * (MR + 2 * MO);   // [W][MR + MO faces, MO dc]
    float4* dcs = faces + MR + MO;
    double* d64 = reinterpret_cast<double*>(reinterpret_cast<float4*>(lds) + W * (MR + 2 * MO)) + wave * MO;
    float* red = reinterpret_cast<float*>(reinterpret_cast<double*>(reinterpret_cast<float4*>(lds) +
                                                                    W * (MR + 2 * MO)) + W * MO);   // [W]
    for (int wg = blockIdx.x; wg < P.n_wg; wg += gridDim.x) {
        const int4 item = P.wg_items[wg];
        const int s = uniform(item.x);
        const int b = uniform(item.y + wave);
        const int t = lane + 1;
        // the state entries of the pose and the multipliers are loaded beside
        // the block's descriptor and the done flag (an empty slot loads a
        // valid pair's values and ignores them)
        const int bq = min(b, item.z - 1), tq = min(t, N);
        PoseInputs<DIM> pin;
        load_pose_state<DIM>(P, P.x + ((size_t)s * (N + 1) + tq) * P.n_s, pin);
        float* zp = P.zeta + (size_t)bq * N + tq - 1;
        const float zeta = *zp;
        float xi[DIM];
#pragma unroll
        for (int r = 0; r < DIM; ++r) xi[r] = P.xi[((size_t)bq * DIM + r) * N + tq - 1];
        const int4 bd = b < item.z ? P.bdesc[b] : int4{0, 0, 0, 0};
        if (P.done[s]) continue;
        const int fr0 = uniform(bd.x), fo0 = uniform(bd.y), yoff = uniform(bd.z);
        const int nr = uniform(bd.w & 0xff), no = uniform((bd.w >> 8) & 0xff), part = uniform(bd.w >> 16);
        // then, beside the faces, the part offset and every row's dual
        // (unconditional loads from clamped rows, all in flight at once)
        load_pose_offset<DIM>(P, part, pin);
        const float* yb = P.y + yoff + (tq - 1);
        float yr[MR], yo[MO];
#pragma unroll
        for (int k = 0; k < MR; ++k) yr[k] = yb[max(0, min(k, nr - 1)) * N];
#pragma unroll
        for (int l = 0; l < MO; ++l) yo[l] = yb[(nr + max(0, min(l, no - 1))) * N];
        const float yg = yb[(nr + no) * N];
        if (b < item.z) {
            if (lane < nr) faces[lane] = P.part_faces[fr0 + lane];
            else if (lane >= MR && lane - MR < no) {
                faces[lane] = P.obs_faces[fo0 + lane - MR];
                dcs[lane - MR] = P.obs_dc[fo0 + lane - MR];
                d64[lane - MR] = P.obs_d64[fo0 + lane - MR];
            }
        }
        __syncthreads();
        float rp = 0.f;
        if (b < item.z && t <= N) {
            Pose<DIM> ps;
            make_pose_v<DIM>(pin.xp, pin.xa, pin.o, ps);
            float Al[DIM] = {}, Sd = 0.f, Sc[DIM] = {};
#pragma unroll
            for (int k = 0; k < MR; ++k) {
                if (k < nr) {
                    const float4 f = faces[k];
                    const float y = yr[k];
                    Al[0] += y * f.x;
                    Al[1] += y * f.y;
                    if (DIM == 3) Al[DIM - 1] += y * f.z;
                }
            }
#pragma unroll
            for (int l = 0; l < MO; ++l) {
                if (l < no) {
                    const float4 f = faces[MR + l];
                    const float y = yo[l];
                    const float dp = face_offset(d64, l, f, dcs[l], ps.pos64, ps.pos, DIM);
                    Sd += dp * y;
                    Sc[0] += f.x * y;
                    Sc[1] += f.y * y;
                    if (DIM == 3) Sc[DIM - 1] += f.z * y;
                }
            }
            const float T = 1.f + Sd + yg;
            *zp = zeta + T;
            rp = T * T;
#pragma unroll
            for (int r = 0; r < DIM; ++r) {
                float acc = Al[r];
#pragma unroll
                for (int m = 0; m < DIM; ++m) acc += ps.R[m * DIM + r] * Sc[m];
                P.xi[((size_t)b * DIM + r) * N + t - 1] = xi[r] + acc;
                rp += acc * acc;
            }
        }
        const float rw = wave_sum(rp);
        if (lane == 0) red[wave] = rw;
        __syncthreads();
        if (threadIdx.x == 0) {
            float a = 0.f;
            for (int w = 0; w < W; ++w) a += red[w];
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

template <int DIM>
struct PairCols {
    int nr, no, fo0;
    const float4* rf;
    const float4* of;
    const double* d64;
    const float4* dc;
    float R[DIM * DIM];
    double pos64[DIM];
    float pos[DIM];
    float cmx;
    __device__ int n() const { return nr + no; }
    __device__ float cmax() const { return cmx; }
    __device__ float cost(int j) const {
        if (j < nr) return 0.f;
        return face_offset(d64, fo0 + j - nr, of[j - nr], dc[fo0 + j - nr], pos64, pos, DIM);
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
    for (int i = 0; i < DIM; ++i) {
        pc.pos64[i] = ps.pos64[i];
        pc.pos[i] = ps.pos[i];
    }
    pc.fo0 = fo0;
    pc.d64 = P.obs_d64;
    pc.dc = P.obs_dc;
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
static void launch_pair_g(const DevProblem& P, int W, int G, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const int nc = P.nc;
    const int nw = pair_waves_per_block(P.N, G);
    const size_t lds = (size_t)W * (MR + 2 * MO) * sizeof(float4) + (size_t)W * MO * sizeof(double) +
                       (size_t)W * nc * 64 * sizeof(float) + 2 * (size_t)W * nw * sizeof(float);
    dim3 blk(64 * W * nw), grd(grid);
    if (G == 4) CADMM_LAUNCH((pair_phase_kernel<DIM, MR, MO, 4>), grd, blk, lds, st, e0, e1, P);
    else if (G == 2) CADMM_LAUNCH((pair_phase_kernel<DIM, MR, MO, 2>), grd, blk, lds, st, e0, e1, P);
    else CADMM_LAUNCH((pair_phase_kernel<DIM, MR, MO, 1>), grd, blk, lds, st, e0, e1, P);
}

bool pair_group_supported(int N, int W, int G)
{
    return (G == 1 || G == 2 || G == 4) && W >= 1 && W * pair_waves_per_block(N, G) <= 8;
}

hipError_t launch_pair_phase(const DevProblem& P, int W, int G, int grid, hipStream_t st, hipEvent_t e0,
                             hipEvent_t e1)
{
    if (!pair_group_supported(P.N, W, G)) return hipErrorInvalidValue;
    switch (pick_variant(P)) {
    case 0: launch_pair_g<2, 4, 16>(P, W, G, grid, st, e0, e1); break;
    case 1: launch_pair_g<2, 8, 32>(P, W, G, grid, st, e0, e1); break;
    case 2: launch_pair_g<3, 6, 24>(P, W, G, grid, st, e0, e1); break;
    case 3: launch_pair_g<3, 8, 32>(P, W, G, grid, st, e0, e1); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mult_phase(const DevProblem& P, int W, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const int v = pick_variant(P);
    if (v < 0) return hipErrorInvalidValue;
    const Variant& vv = kVariants[v];
    const size_t lds = (size_t)W * ((vv.mr + 2 * vv.mo) * sizeof(float4) + vv.mo * sizeof(double) + sizeof(float));
    dim3 blk(64 * W), grd(grid);
    switch (v) {
    case 0: CADMM_LAUNCH((mult_phase_kernel<2, 4, 16>), grd, blk, lds, st, e0, e1, P); break;
    case 1: CADMM_LAUNCH((mult_phase_kernel<2, 8, 32>), grd, blk, lds, st, e0, e1, P); break;
    case 2: CADMM_LAUNCH((mult_phase_kernel<3, 6, 24>), grd, blk, lds, st, e0, e1, P); break;
    case 3: CADMM_LAUNCH((mult_phase_kernel<3, 8, 32>), grd, blk, lds, st, e0, e1, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_residual(const DevProblem& P, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    CADMM_LAUNCH(residual_kernel, dim3(P.n_scen), dim3(64), 0, st, e0, e1, P);
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

}  // namespace cadmm
