// Shared solvers of the gfx950 collision-avoidance kernels (arXiv 2406.07048):
// the dual semismooth Newton method for the dual-update QP (Sec. IV-C eq.
// const_least_square with the proximal term) and the revised simplex for
// the scale LP (Sec. III-A eq. scale_opt through its dual, Sec. III-B eq.
// scale_opt_dual). Both take their rows / columns from a source class, so
// the ADMM kernels (structured pair data) and the stateless batch kernels
// (rows from memory) share the iteration.
#pragma once
#include "cadmm_device.h"

#include <float.h>
#include <math.h>

namespace cadmm {

// ------------------------------------------------------------------------
// semismooth Newton on the concave dual, shared by both row sources.
// Returns the sweeps used, or -1 if the budget ran out (z is still the last
// iterate, whose primal y is within the Newton region in practice), or
// kNewtonPaused when stop_at sweeps were reached first: the state then holds
// the point to resume from, and the resumed solve takes exactly the iterates
// of an uninterrupted one.
// ------------------------------------------------------------------------

struct NewtonState {
    float gprev = FLT_MAX;   // gradient of the previous sweep (stall test)
    float al_prev = 1.f;     // step accepted by the previous sweep
    int it = 0;              // sweeps done
};
constexpr int kNewtonPaused = -2;

template <int NV, class Rows>
__device__ int dual_newton(const Rows& rows, float (&z)[NV], int max_sweeps, float gtol, NewtonState& S,
                           int stop_at)
{
    float& gprev = S.gprev;
    float& al_prev = S.al_prev;
    for (; S.it < max_sweeps; ++S.it) {
        if (S.it >= stop_at) return kNewtonPaused;
        const int it = S.it;
        float g[NV], H[NV * NV], sc;
        rows.template pass<true>(z, g, H, sc);
        float gmax = 0.f, zmax = 0.f;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            gmax = fmaxf(gmax, fabsf(g[i]));
            zmax = fmaxf(zmax, fabsf(z[i]));
        }
        // converged (gradient at gtol of its scale), or stalled: iterates that
        // stop improving below 5e-7 sc sit at the FP32 floor of the gradient
        // (about 3e-8 to 1.3e-7 sc at the optimum of C2/C3 pairs, measured in
        // an FP32 emulation against the FP64 active-set solution); iterating
        // on only spends the budget. A looser stall level (4e-6 sc) let pairs
        // with slow line searches stop with scaled dual errors up to 2e-5;
        // at 5e-7 the same pairs reach 1e-7 for 3% more row passes. Inside
        // the ADMM loop gtol = 1e-7, near the floor: each solve starts from
        // the previous iteration's duals, and with 1e-6 the next iteration
        // needed more sweeps (C3 pair phase 124 -> 90 us). Cold-started
        // stateless batches use 1e-6 (scaled dual error <= 3.4e-6 on C3 pairs).
        if (gmax <= gtol * sc || (gmax <= 5e-7f * sc && gmax >= 0.7f * gprev)) return it;
        gprev = gmax;
        float dz[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) dz[i] = g[i];
        chol_solve<NV>(H, dz);
        // After a short step the direction is often steered by rows whose
        // dual is about to switch on or off; they stop it at the first kink
        // every sweep. Re-solve with the generalised Hessian of every row
        // active at z or at the full step z + dz and take that direction when
        // it is still an ascent direction. (The Hessian of the full step's
        // active set alone let pairs with two such rows zig-zag between the
        // kinks at half the gradient per ten sweeps until the budget ran out:
        // scaled dual errors of 1e-4, reproduced in an FP32 emulation of this
        // solver; with the union none remain.)
        if (al_prev < 0.1f) {
            float zt[NV], gt[NV], Ht[NV * NV], sct, dz2[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) zt[i] = z[i] + dz[i];
            rows.template pass<true, true>(z, gt, Ht, sct, zt);
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
        // directional derivative of the dual along dz at step al; the trial
        // with the smallest gradient is kept as a fallback
        float best_al = 0.f, best_g = gmax;
        auto dphi = [&](float al) {
            float zt[NV], gt[NV], Hd[NV * NV], sct;
#pragma unroll
            for (int i = 0; i < NV; ++i) zt[i] = z[i] + al * dz[i];
            rows.template pass<false>(zt, gt, Hd, sct);
            float d = 0.f, gm = 0.f;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                d += dz[i] * gt[i];
                gm = fmaxf(gm, fabsf(gt[i]));
            }
            if (gm < best_g) {
                best_g = gm;
                best_al = al;
            }
            return d;
        };
        float al = 1.f;
        const float d1 = dphi(1.f);
        if (d1 < -1e-3f * d0) {
            // Illinois regula falsi on the decreasing piecewise-linear dphi
            float lo = 0.f, hi = 1.f, flo = d0, fhi = d1;
            int side = 0;
            for (int ls = 0; ls < 6; ++ls) {
                al = (lo * (-fhi) + hi * flo) * __builtin_amdgcn_rcpf(flo - fhi);
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
            // no step along dz passes the sign test (the directional
            // derivative is at its FP32 floor): take the trial that lowered
            // the gradient most, else z cannot be improved along dz and every
            // further sweep would repeat this one exactly
            if (al == 0.f) {
                if (best_al == 0.f) return it + 1;
                al = best_al;
            }
        }
#pragma unroll
        for (int i = 0; i < NV; ++i) z[i] += al * dz[i];
        al_prev = al;
    }
    return -1;
}

template <int NV, class Rows>
__device__ int dual_newton(const Rows& rows, float (&z)[NV], int max_sweeps, float gtol)
{
    NewtonState S;
    return dual_newton<NV>(rows, z, max_sweeps, gtol, S, 0x7fffffff);
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
}  // namespace cadmm
