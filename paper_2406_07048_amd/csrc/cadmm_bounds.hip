// State and input bounds of the trajectory QP (Sec. IV-A eq. MPC_opt_origin,
// its state and control rows: the indicator IC_0 of eq. ADMM_Lagrangian
// taken in full in the state update of Sec. IV-B eq. ADMM_state_updates).
//
// The trajectory kernel leaves the unconstrained minimiser of the iteration's
// QP in x, u. Where it breaks a bound, this kernel (one wavefront per
// scenario) moves it to the bounded minimiser by the dual active-set method
// of Goldfarb and Idnani (1983): from the unconstrained point, take the most
// violated bound p, move along the direction that keeps the active bounds
// satisfied while p's multiplier grows, and drop an active bound whose
// multiplier reaches zero first. The QP's inverse Hessian (on the subspace
// the dynamics leave free) is applied through a Riccati factorisation of the
// same stage Hessians: G^{-1} e_v is the LQ solution for a unit linear cost
// on the variable v with zero initial state and no offsets, one backward
// sweep from v's step down and one forward rollout. The directions of the
// active bounds live in global memory (one slot each), the Cholesky factor
// of N_A^T G^{-1} N_A in LDS.
#include "cadmm_internal.h"
#include "cadmm.h"

#include <float.h>

namespace cadmm {

namespace {

constexpr int kBlock = 64;

__device__ __forceinline__ void wave_argmin_b(float& v, int& key)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float ov = __shfl_xor(v, o, 64);
        const int ok = __shfl_xor(key, o, 64);
        if (ov < v || (ov == v && ok < key)) { v = ov; key = ok; }
    }
}

__device__ __forceinline__ float wave_sum_b(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Variables of one scenario: states x_t (t = 1..N) at v = (t-1) ns + i, then
// inputs u_t (t = 0..N-1) at N ns + t nu + j. Bound id 2 v (lower) or 2 v + 1
// (upper).
struct Vars {
    int ns, nu, N;
    __device__ int count() const { return N * (ns + nu); }
    __device__ bool is_state(int v) const { return v < N * ns; }
};

}  // namespace

// Bounded trajectory QP; see the file comment. x, u hold the unconstrained
// minimiser on entry and the bounded one on exit; bstat[s] receives the
// number of active bounds, -1 (bounds infeasible), -2 (more active bounds
// than slots) or -3 (step cap), the iterate then left at the last point.
template <int NS, int NU>
__global__ void __launch_bounds__(kBlock) traj_bounds_kernel(DevProblem P, int obstacle_free)
{
    constexpr int NMAX = CADMM_MAX_N;
    constexpr int SL = kBoundSlots;
    __shared__ float Kf[NMAX][NU * NS];     // gains K_t
    __shared__ float Qi[NMAX][NU * NU];     // (R + B^T P B)^{-1} of step t
    __shared__ float Pm[NS * NS], PA[NS * NS], PB[NS * NU], Quu[NU * NU], Qux[NU * NS];
    __shared__ float xs[(NMAX + 1) * NS];   // x_t, t = 0..N (row t at t * ns)
    __shared__ float us[NMAX * NU];
    __shared__ float wl[NMAX * (NS + NU)];  // direction G^{-1} n_p in variable order
    __shared__ float kk[NMAX * NU];         // feedforward of the direction sweep
    __shared__ float pv[NS], bp[NU], dx[NS], du[NU];
    __shared__ float LM[SL * SL];           // Cholesky factor of N_A^T G^{-1} N_A (row-major, lower)
    __shared__ int av[SL];                  // active bound ids
    __shared__ float lam[SL], rr[SL], ym[SL];
    __shared__ unsigned char act[NMAX * (NS + NU)];   // 0 free, 1 lower active, 2 upper active
    __shared__ int pidx[NS];
    // the models of the steps in LDS (every sweep reads them step by step):
    // one time-invariant model, or up to MCS per-step models
    constexpr int MCS = NS <= 4 ? NMAX : 16;
    __shared__ float Mc[MCS * (NS * NS + NS * NU)];

    const int s = blockIdx.x;
    if (!obstacle_free && P.done[s]) return;
    const int lane = threadIdx.x;
    const int ns = P.n_s, nu = P.n_u, N = P.N, nc = P.nc, nq = P.nq;
    const Vars V{ns, nu, N};
    const int nv = V.count();
    // the models the trajectory kernel used: the iteration's linearisation
    // for a nonlinear model, else the given linear models (stride 0: shared)
    const bool sqp = P.model != 0 && !obstacle_free;
    const float* Ag = sqp ? P.A_lin + (size_t)s * N * ns * ns : P.A_dyn + (size_t)s * P.dyn_ss * ns * ns;
    const float* Bg = sqp ? P.B_lin + (size_t)s * N * ns * nu : P.B_dyn + (size_t)s * P.dyn_ss * ns * nu;
    const int mts = sqp ? 1 : P.dyn_ts;
    const int msz = ns * ns + ns * nu;               // floats of one cached model
    const int n_mod = mts == 0 ? 1 : N;
    const bool cached = n_mod <= MCS;
    if (cached) {
        for (int e = threadIdx.x; e < n_mod * msz; e += kBlock) {
            const int t = e / msz, q = e % msz;
            Mc[e] = q < ns * ns ? Ag[(size_t)t * mts * ns * ns + q] : Bg[(size_t)t * mts * ns * nu + (q - ns * ns)];
        }
    }
    auto Am = [&](int t, int i, int j) {
        return cached ? Mc[(mts ? t : 0) * msz + i * ns + j] : Ag[(size_t)t * mts * ns * ns + i * ns + j];
    };
    auto Bm = [&](int t, int i, int j) {
        return cached ? Mc[(mts ? t : 0) * msz + ns * ns + i * nu + j] : Bg[(size_t)t * mts * ns * nu + i * nu + j];
    };
    float* xo = P.x + (size_t)s * (N + 1) * ns;
    float* uo = P.u + (size_t)s * N * nu;
    auto zval = [&](int v) -> float {
        return V.is_state(v) ? xs[(v / ns + 1) * ns + v % ns] : us[v - N * ns];
    };
    auto lo_of = [&](int v) -> float { return V.is_state(v) ? P.xlo[v % ns] : P.ulo[(v - N * ns) % nu]; };
    auto hi_of = [&](int v) -> float { return V.is_state(v) ? P.xhi[v % ns] : P.uhi[(v - N * ns) % nu]; };

    for (int e = lane; e < (N + 1) * ns; e += kBlock) xs[e] = xo[e];
    for (int e = lane; e < N * nu; e += kBlock) us[e] = uo[e];
    for (int v = lane; v < nv; v += kBlock) act[v] = 0;
    if (lane < NS) {
        int a_of = -1;
        for (int a = 0; a < nq; ++a) {
            const int qa = a < P.dim ? P.pos_idx[a] : P.att_idx[a - P.dim];
            if (qa == lane && lane < ns) a_of = a;
        }
        pidx[lane] = a_of;
    }
    __syncthreads();

    // most violated free bound: (slack, id); slack +inf if none
    auto worst_bound = [&](float& sl, int& id) {
        sl = INFINITY;
        id = 0x7fffffff;
        for (int v = lane; v < nv; v += kBlock) {
            if (act[v]) continue;
            const float z = zval(v), lo = lo_of(v), hi = hi_of(v);
            if (lo > -INFINITY) {
                const float d = z - lo;
                if (d < -2e-6f * fmaxf(1.f, fabsf(lo)) && d < sl) { sl = d; id = 2 * v; }
            }
            if (hi < INFINITY) {
                const float d = hi - z;
                if (d < -2e-6f * fmaxf(1.f, fabsf(hi)) && d < sl) { sl = d; id = 2 * v + 1; }
            }
        }
        wave_argmin_b(sl, id);
    };
    float sl;
    int pid;
    worst_bound(sl, pid);
    if (!(sl < INFINITY)) {
        if (lane == 0) {
            P.bstat[s] = 0;
            P.bprev[(size_t)s * (SL + 1)] = 0;
        }
        return;
    }

    // 1. Riccati factorisation of the stage Hessians: H_t = 2 Q_s plus the
    //    pose block of the pair terms (t = 1..N), 2 Q_u for the inputs.
    auto Hst = [&](int t, int i, int j) -> float {   // t = 1..N
        float h = 2.f * P.Q_s[i * ns + j];
        if (!obstacle_free && pidx[i] >= 0 && pidx[j] >= 0) {
            const int a = min(pidx[i], pidx[j]), b = max(pidx[i], pidx[j]);
            h += P.hq_b[((size_t)s * N + (t - 1)) * nc + a * nq - a * (a - 1) / 2 + (b - a)];
        }
        return h;
    };
    for (int e = lane; e < ns * ns; e += kBlock) Pm[e] = Hst(N, e / ns, e % ns);
    __syncthreads();
    for (int t = N - 1; t >= 0; --t) {
        for (int e = lane; e < ns * (ns + nu); e += kBlock) {
            if (e < ns * ns) {
                const int i = e / ns, j = e % ns;
                float acc = 0.f;
                for (int r = 0; r < ns; ++r) acc += Pm[i * ns + r] * Am(t, r, j);
                PA[e] = acc;
            } else {
                const int f = e - ns * ns, i = f / nu, j = f % nu;
                float acc = 0.f;
                for (int r = 0; r < ns; ++r) acc += Pm[i * ns + r] * Bm(t, r, j);
                PB[f] = acc;
            }
        }
        __syncthreads();
        for (int e = lane; e < nu * (nu + ns); e += kBlock) {
            if (e < nu * nu) {
                const int i = e / nu, j = e % nu;
                float acc = 2.f * P.Q_u[i * nu + j];
                for (int r = 0; r < ns; ++r) acc += Bm(t, r, i) * PB[r * nu + j];
                Quu[e] = acc;
            } else {
                const int f = e - nu * nu, i = f / ns, j = f % ns;
                float acc = 0.f;
                for (int r = 0; r < ns; ++r) acc += Bm(t, r, i) * PA[r * ns + j];
                Qux[f] = acc;
            }
        }
        __syncthreads();
        // the small inverse by Gauss-Jordan on the SPD Quu (padded with the
        // identity), by lane 0, into LDS; then the gains from it
        if (lane == 0) {
            float Wm[NU][2 * NU];
#pragma unroll
            for (int i = 0; i < NU; ++i)
#pragma unroll
                for (int j = 0; j < 2 * NU; ++j) {
                    float v = 0.f;
                    if (j < NU) v = (i < nu && j < nu) ? Quu[i * nu + j] : (i == j ? 1.f : 0.f);
                    else v = (j - NU == i) ? 1.f : 0.f;
                    Wm[i][j] = v;
                }
#pragma unroll
            for (int c = 0; c < NU; ++c) {
                const float ip = 1.f / Wm[c][c];
#pragma unroll
                for (int j = 0; j < 2 * NU; ++j) Wm[c][j] *= ip;
#pragma unroll
                for (int i = 0; i < NU; ++i) {
                    if (i == c) continue;
                    const float f = Wm[i][c];
#pragma unroll
                    for (int j = 0; j < 2 * NU; ++j) Wm[i][j] -= f * Wm[c][j];
                }
            }
#pragma unroll
            for (int i = 0; i < NU; ++i)
#pragma unroll
                for (int j = 0; j < NU; ++j) Qi[t][i * NU + j] = Wm[i][NU + j];
        }
        __syncthreads();
        for (int e = lane; e < nu * ns; e += kBlock) {
            const int j = e / ns, i = e % ns;
            float acc = 0.f;
            for (int m = 0; m < nu; ++m) acc -= Qi[t][j * NU + m] * Qux[m * ns + i];
            Kf[t][j * NS + i] = acc;
        }
        __syncthreads();
        if (t >= 1) {
            // P_t = H_t + A^T P A + Qux^T K, symmetrised
            for (int e = lane; e < ns * ns; e += kBlock) {
                const int i = e / ns, j = e % ns;
                if (j < i) continue;
                float a1 = 0.f, a2 = 0.f;
                for (int r = 0; r < ns; ++r) {
                    a1 += Am(t, r, i) * PA[r * ns + j];
                    a2 += Am(t, r, j) * PA[r * ns + i];
                }
                for (int m = 0; m < nu; ++m) {
                    a1 += Qux[m * ns + i] * Kf[t][m * NS + j];
                    a2 += Qux[m * ns + j] * Kf[t][m * NS + i];
                }
                const float h = Hst(t, i, j);
                const float v = h + 0.5f * (a1 + a2);
                Pm[i * ns + j] = v;
                Pm[j * ns + i] = v;
            }
            __syncthreads();
        }
    }

    // 2. the directions of the bounds active at the end of the previous
    //    trajectory QP (usually the ones this one needs), all in one sweep
    //    pair: the recursion of the single sweep below run on k right-hand
    //    sides at once, in the same order of operations (bitwise the same
    //    directions). The backward pass leaves the feedforward of step t in
    //    the input part of each direction's slot, which the forward pass
    //    overwrites with the inputs.
    __shared__ int cid[SL];                 // bound ids of the precomputed directions
    float* Wc = P.bW + ((size_t)P.n_scen + s) * SL * nv;   // their slots
    int nC = P.bprev[(size_t)s * (SL + 1)];
    if (nC < 0 || nC > SL) nC = 0;
    if (lane < nC) cid[lane] = P.bprev[(size_t)s * (SL + 1) + 1 + lane];
    __syncthreads();
    if (nC > 0) {
        float* Pk = LM;                      // [ns][SL], then [ns][SL] (double buffer)
        float* Pk2 = LM + NS * SL;
        float* BK = LM + 2 * NS * SL;        // [nu][SL]
        auto dvar = [&](int j) { return cid[j] >> 1; };
        auto dsg = [&](int j) { return (cid[j] & 1) ? -1.f : 1.f; };
        // p_N: the state directions at x_N
        for (int e = lane; e < ns * nC; e += kBlock) {
            const int i = e / nC, j = e % nC, v = dvar(j);
            Pk[i * SL + j] = (V.is_state(v) && v / ns + 1 == N && v % ns == i) ? -dsg(j) : 0.f;
        }
        __syncthreads();
        for (int t = N - 1; t >= 0; --t) {
            for (int e = lane; e < nu * nC; e += kBlock) {
                const int c = e / nC, j = e % nC;
                float acc = 0.f;
                for (int r = 0; r < ns; ++r) acc += Bm(t, r, c) * Pk[r * SL + j];
                BK[c * SL + j] = acc;
            }
            __syncthreads();
            for (int e = lane; e < nu * nC; e += kBlock) {
                const int c = e / nC, j = e % nC, v = dvar(j);
                float acc = 0.f;
                for (int m = 0; m < nu; ++m) acc -= Qi[t][c * NU + m] * BK[m * SL + j];
                if (!V.is_state(v) && (v - N * ns) / nu == t) acc += dsg(j) * Qi[t][c * NU + (v - N * ns) % nu];
                Wc[(size_t)j * nv + N * ns + t * nu + c] = acc;
            }
            if (t >= 1) {
                for (int e = lane; e < ns * nC; e += kBlock) {
                    const int i = e / nC, j = e % nC, v = dvar(j);
                    float pn = 0.f;
                    for (int r = 0; r < ns; ++r) pn += Am(t, r, i) * Pk[r * SL + j];
                    for (int m = 0; m < nu; ++m) pn += Kf[t][m * NS + i] * BK[m * SL + j];
                    if (!V.is_state(v) && (v - N * ns) / nu == t) pn += -dsg(j) * Kf[t][((v - N * ns) % nu) * NS + i];
                    if (V.is_state(v) && v / ns + 1 == t && v % ns == i) pn += -dsg(j);
                    Pk2[i * SL + j] = pn;
                }
            }
            __syncthreads();
            if (t >= 1)
                for (int e = lane; e < ns * nC; e += kBlock) Pk[(e / nC) * SL + e % nC] = Pk2[(e / nC) * SL + e % nC];
            __threadfence_block();
            __syncthreads();
        }
        // forward: dx_0 = 0
        float* DX = Pk;
        float* DX2 = Pk2;
        for (int e = lane; e < ns * nC; e += kBlock) DX[(e / nC) * SL + e % nC] = 0.f;
        __syncthreads();
        for (int t = 0; t < N; ++t) {
            for (int e = lane; e < nu * nC; e += kBlock) {
                const int c = e / nC, j = e % nC;
                float* slot = Wc + (size_t)j * nv + N * ns + t * nu + c;
                float acc = *slot;
                for (int i = 0; i < ns; ++i) acc += Kf[t][c * NS + i] * DX[i * SL + j];
                BK[c * SL + j] = acc;
                *slot = acc;
            }
            __syncthreads();
            for (int e = lane; e < ns * nC; e += kBlock) {
                const int i = e / nC, j = e % nC;
                float xn = 0.f;
                for (int r = 0; r < ns; ++r) xn += Am(t, i, r) * DX[r * SL + j];
                for (int m = 0; m < nu; ++m) xn += Bm(t, i, m) * BK[m * SL + j];
                DX2[i * SL + j] = xn;
                Wc[(size_t)j * nv + t * ns + i] = xn;
            }
            __syncthreads();
            for (int e = lane; e < ns * nC; e += kBlock) DX[(e / nC) * SL + e % nC] = DX2[(e / nC) * SL + e % nC];
            __syncthreads();
        }
        __threadfence_block();
        __syncthreads();
    }

    // 3. dual active-set steps
    float* W = P.bW + (size_t)s * SL * nv;     // slot i: the direction of active bound i
    int nA = 0, status = 0, steps = 0;
    const int cap = 4 * SL + 2 * nv;
    float lam_p = 0.f;
    bool have_dir = false;
    while (true) {
        if (!have_dir) {
            if (nA > 0 || steps > 0) worst_bound(sl, pid);
            if (!(sl < INFINITY)) break;
            lam_p = 0.f;
            // a direction of the previous active set
            const unsigned long long hit = __ballot(lane < nC && cid[lane] == pid);
            if (hit) {
                const int j = __builtin_ctzll(hit);
                for (int v = lane; v < nv; v += kBlock) wl[v] = Wc[(size_t)j * nv + v];
                __syncthreads();
                have_dir = true;
                continue;
            }
            // direction w = sg G^{-1} e_v: the LQ solution for the linear cost
            // -sg e_v (zero initial state, no offsets)
            const int v = pid >> 1;
            const float sg = (pid & 1) ? -1.f : 1.f;
            int t0;   // last step whose feedforward may be nonzero
            for (int e = lane; e < N * nu; e += kBlock) kk[e] = 0.f;
            __syncthreads();
            if (V.is_state(v)) {
                const int ts = v / ns + 1, i = v % ns;
                if (lane < ns) pv[lane] = lane == i ? -sg : 0.f;
                t0 = ts - 1;
            } else {
                const int ts = (v - N * ns) / nu, j = (v - N * ns) % nu;
                if (lane < nu) kk[ts * nu + lane] = sg * Qi[ts][lane * NU + j];
                if (lane < ns) pv[lane] = -sg * Kf[ts][j * NS + lane];
                t0 = ts - 1;
            }
            __syncthreads();
            for (int t = t0; t >= 0; --t) {
                if (lane < nu) {
                    float acc = 0.f;
                    for (int r = 0; r < ns; ++r) acc += Bm(t, r, lane) * pv[r];
                    bp[lane] = acc;
                }
                __syncthreads();
                float pn = 0.f;
                if (lane < nu) {
                    float acc = 0.f;
                    for (int m = 0; m < nu; ++m) acc -= Qi[t][lane * NU + m] * bp[m];
                    kk[t * nu + lane] = acc;
                }
                if (lane < ns && t >= 1) {
                    for (int r = 0; r < ns; ++r) pn += Am(t, r, lane) * pv[r];
                    for (int m = 0; m < nu; ++m) pn += Kf[t][m * NS + lane] * bp[m];
                }
                __syncthreads();
                if (lane < ns && t >= 1) pv[lane] = pn;
                __syncthreads();
            }
            // rollout from dx_0 = 0
            if (lane < ns) dx[lane] = 0.f;
            __syncthreads();
            for (int t = 0; t < N; ++t) {
                if (lane < nu) {
                    float acc = kk[t * nu + lane];
                    for (int i = 0; i < ns; ++i) acc += Kf[t][lane * NS + i] * dx[i];
                    du[lane] = acc;
                    wl[N * ns + t * nu + lane] = acc;
                }
                __syncthreads();
                float xn = 0.f;
                if (lane < ns) {
                    for (int r = 0; r < ns; ++r) xn += Am(t, lane, r) * dx[r];
                    for (int m = 0; m < nu; ++m) xn += Bm(t, lane, m) * du[m];
                }
                __syncthreads();
                if (lane < ns) {
                    dx[lane] = xn;
                    wl[t * ns + lane] = xn;
                }
                __syncthreads();
            }
            have_dir = true;
        }
        if (++steps > cap) { status = -3; break; }
        const int vp = pid >> 1;
        const float sgp = (pid & 1) ? -1.f : 1.f;
        const float pp = sgp * wl[vp];
        // r = M^{-1} m, m_i = n_i^T w_p: forward (y = L^{-1} m) and backward
        // substitution, lane i holding row i
        float acc = 0.f;
        int vi = 0;
        float sgi = 0.f;
        if (lane < nA) {
            vi = av[lane] >> 1;
            sgi = (av[lane] & 1) ? -1.f : 1.f;
            acc = sgi * wl[vi];
        }
        for (int j = 0; j < nA; ++j) {
            const float yj = __shfl(acc, j, 64) / LM[j * SL + j];
            if (lane == j) acc = yj;
            else if (lane > j && lane < nA) acc -= LM[lane * SL + j] * yj;
        }
        const float yv = acc;     // L^{-1} m
        if (lane < nA) ym[lane] = yv;
        for (int j = nA - 1; j >= 0; --j) {
            const float rj = __shfl(acc, j, 64) / LM[j * SL + j];
            if (lane == j) acc = rj;
            else if (lane < j) acc -= LM[j * SL + lane] * rj;
        }
        if (lane < nA) rr[lane] = acc;
        __syncthreads();
        // n_p^T d, d = w_p - sum_i r_i w_i
        float dnp = 0.f;
        if (lane < nA) dnp = rr[lane] * W[(size_t)lane * nv + vp];
        const float dn = sgp * (wl[vp] - wave_sum_b(dnp));
        // partial step: the first active multiplier to reach zero
        float t2 = INFINITY;
        int kb = 0x7fffffff;
        if (lane < nA && rr[lane] > 0.f) { t2 = lam[lane] / rr[lane]; kb = lane; }
        wave_argmin_b(t2, kb);
        const float sp = (pid & 1) ? hi_of(vp) - zval(vp) : zval(vp) - lo_of(vp);
        const bool dependent = !(dn > 1e-5f * pp);
        if (dependent && !(t2 < INFINITY)) { status = -1; break; }
        const float t1 = dependent ? INFINITY : -sp / dn;
        const float tt = fminf(t1, t2);
        if (!dependent) {
            for (int v = lane; v < nv; v += kBlock) {
                float d = wl[v];
                for (int i = 0; i < nA; ++i) d -= rr[i] * W[(size_t)i * nv + v];
                if (V.is_state(v)) xs[(v / ns + 1) * ns + v % ns] += tt * d;
                else us[v - N * ns] += tt * d;
            }
        }
        if (lane < nA) lam[lane] -= tt * rr[lane];
        lam_p += tt;
        __syncthreads();
        if (t1 <= t2) {
            // full step: p joins the active set; the new row of the factor is
            // y = L^{-1} m with diagonal sqrt(n_p^T d)
            if (nA == SL) { status = -2; break; }
            for (int v = lane; v < nv; v += kBlock) W[(size_t)nA * nv + v] = wl[v];
            if (lane < nA) LM[nA * SL + lane] = ym[lane];
            if (lane == 0) {
                LM[nA * SL + nA] = sqrtf(dn);
                av[nA] = pid;
                lam[nA] = lam_p;
                act[vp] = (pid & 1) ? 2 : 1;
            }
            ++nA;
            have_dir = false;
            __threadfence_block();
            __syncthreads();
            continue;
        }
        // partial step: drop bound kb (the last one moves into its slot) and
        // refactor N_A^T G^{-1} N_A
        const int last = nA - 1;
        if (lane == 0) {
            act[av[kb] >> 1] = 0;
            av[kb] = av[last];
            lam[kb] = lam[last];
        }
        if (kb != last)
            for (int v = lane; v < nv; v += kBlock) W[(size_t)kb * nv + v] = W[(size_t)last * nv + v];
        nA = last;
        __threadfence_block();
        __syncthreads();
        // M_ij = sg_i sg_j w_j[v_i], lane i owning row i
        for (int j = 0; j < nA; ++j) {
            // diagonal
            if (lane == j) {
                const int vj = av[j] >> 1;
                const float sj = (av[j] & 1) ? -1.f : 1.f;
                float d = sj * W[(size_t)j * nv + vj];
                for (int k2 = 0; k2 < j; ++k2) d -= LM[j * SL + k2] * LM[j * SL + k2];
                LM[j * SL + j] = sqrtf(fmaxf(d, 1e-30f));
            }
            __syncthreads();
            if (lane > j && lane < nA) {
                const int vl = av[lane] >> 1;
                const float sgl = (av[lane] & 1) ? -1.f : 1.f;
                // n_l^T w_j (w_j carries its own sign)
                float m = sgl * W[(size_t)j * nv + vl];
                for (int k2 = 0; k2 < j; ++k2) m -= LM[lane * SL + k2] * LM[j * SL + k2];
                LM[lane * SL + j] = m / LM[j * SL + j];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int e = lane + ns; e < (N + 1) * ns; e += kBlock) xo[e] = xs[e];
    for (int e = lane; e < N * nu; e += kBlock) uo[e] = us[e];
    if (lane == 0) P.bstat[s] = status < 0 ? status : nA;
    // the final active set, whose directions the next trajectory QP computes first
    const int keep = status < 0 ? 0 : nA;
    if (lane < keep) P.bprev[(size_t)s * (SL + 1) + 1 + lane] = av[lane];
    if (lane == 0) P.bprev[(size_t)s * (SL + 1)] = keep;
}

bool bounds_supported(int n_s, int n_u) { return n_s <= 12 && n_u <= 4; }

hipError_t launch_traj_bounds(const DevProblem& P, int obstacle_free, hipStream_t st, hipEvent_t ev1)
{
    const dim3 g(P.n_scen), b(kBlock);
    if (P.n_s <= 4 && P.n_u <= 2) {
        if (ev1) hipExtLaunchKernelGGL((traj_bounds_kernel<4, 2>), g, b, 0, st, nullptr, ev1, 0, P, obstacle_free);
        else hipLaunchKernelGGL((traj_bounds_kernel<4, 2>), g, b, 0, st, P, obstacle_free);
    } else {
        if (ev1) hipExtLaunchKernelGGL((traj_bounds_kernel<12, 4>), g, b, 0, st, nullptr, ev1, 0, P, obstacle_free);
        else hipLaunchKernelGGL((traj_bounds_kernel<12, 4>), g, b, 0, st, P, obstacle_free);
    }
    return hipGetLastError();
}

}  // namespace cadmm
