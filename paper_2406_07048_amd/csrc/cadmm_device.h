// Device helpers shared by the forward and reverse kernels of the gfx950
// ADMM collision-avoidance library: small register solves, wave sums,
// the pose of a robot part and the FP64 face offsets. Device code only.
#pragma once
#include "cadmm_internal.h"

#include <float.h>
#include <math.h>

namespace cadmm {

// ------------------------------------------------------------------------
// small dense helpers (fully unrolled, registers only)
// ------------------------------------------------------------------------

// In-place Cholesky solve of an SPD system H x = g (H full NV x NV). The
// pivots use v_rsq_f32 (about 1 ulp) and the factor keeps 1 / l_jj on its
// diagonal, so the factorisation and both substitutions multiply instead of
// running IEEE square roots and divisions (each an instruction sequence of
// its own, together most of a small Newton step's VALU work).
template <int NV>
__device__ __forceinline__ void chol_solve(float (&H)[NV * NV], float (&g)[NV])
{
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        float s = H[j * NV + j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= H[j * NV + k] * H[j * NV + k];
        const float iL = __builtin_amdgcn_rsqf(fmaxf(s, 1e-30f));
        H[j * NV + j] = iL;
#pragma unroll
        for (int i = j + 1; i < NV; ++i) {
            float t = H[i * NV + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= H[i * NV + k] * H[j * NV + k];
            H[i * NV + j] = t * iL;
        }
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        float s = g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= H[i * NV + k] * g[k];
        g[i] = s * H[i * NV + i];
    }
#pragma unroll
    for (int i = NV - 1; i >= 0; --i) {
        float s = g[i];
#pragma unroll
        for (int k = i + 1; k < NV; ++k) s -= H[k * NV + i] * g[k];
        g[i] = s * H[i * NV + i];
    }
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lane groups of G = 1, 2 or 4 consecutive lanes (aligned within a quad).
// quad_perm [1,0,3,2] exchanges lanes 2i and 2i+1, [2,3,0,1] lanes i and
// i^2; both stay inside a quad, so groups never read another group's lanes.
// Every DPP move here sets bound_ctrl: each of these patterns reads only
// lanes that exist, so it changes no value, and it lets the compiler fold the
// move into the add or multiply that consumes it (v_add_f32_dpp: 80 fewer
// instructions in the 2D pair kernel with four lanes per pair).
__device__ __forceinline__ float dpp_xor1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true));
}

__device__ __forceinline__ float dpp_xor2(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, true));
}

__device__ __forceinline__ int dpp_xor1_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_xor2_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); }

// Within each row of 16 lanes: a rotation of the row by R lanes (row_ror).

template <int R>
__device__ __forceinline__ float row_ror(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + R, 0xF, 0xF, true));
}


// Sum over a lane group. Every lane of the group gets the bitwise same value
// (pairwise sums in the same order: a + b = b + a exactly).
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (G >= 2) v += dpp_xor1(v);
    if constexpr (G >= 4) v += dpp_xor2(v);
    return v;
}

// ------------------------------------------------------------------------
// pose: R(s), dR/d(attitude), part centre pos_i = rho(s) + R o_i
// ------------------------------------------------------------------------

template <int DIM>
struct Pose {
    static constexpr int NATT = DIM == 2 ? 1 : 3;
    static constexpr int NQ = DIM + NATT;
    float R[DIM * DIM];
    float dR[NATT * DIM * DIM];
    float pos[DIM];
    double pos64[DIM];   // the same centre in FP64 (the state entries are exact in it)
    float q[NQ];   // pose coordinates (position, attitude) of the state
};

// Face offset of an obstacle face in the part frame, d'_l = d_l - c_l.pos.
// d_l and c_l.pos are world-frame numbers of the size of the scene while
// d'_l is of the size of the clearance, so FP32 would lose most of its
// digits to cancellation. Formed in FP64 from the FP64 offset d64, the FP32
// normal f and the FP64 part centre, plus the normal's rounding dc = c_l -
// (float)c_l (stored in FP32, |dc| <= 2^-24 |c_l|) times the FP32 centre:
// without that term the rounded normal alone leaves 6e-8 |pos| (6e-6 m at
// 100 m); with it the error is about 2^-48 |pos|.
__device__ __forceinline__ float face_offset(const double* d64, int face, const float4& f, const float4& dc,
                                             const double* pos64, const float* pos, int dim)
{
    double acc = d64[face] - (double)f.x * pos64[0] - (double)f.y * pos64[1];
    float corr = dc.x * pos[0] + dc.y * pos[1];
    if (dim == 3) {
        acc -= (double)f.z * pos64[2];
        corr += dc.z * pos[2];
    }
    return (float)(acc - (double)corr);
}

// The pose from the state's position entries xp, attitude entries xa and the
// part's offset o (values already loaded; see make_pose).
template <int DIM>
__device__ __forceinline__ void make_pose_v(const float (&xp)[DIM], const float (&xa)[Pose<DIM>::NATT],
                                            const float (&o)[3], Pose<DIM>& ps)
{
    if constexpr (DIM == 2) {
        const float th = xa[0];
        float s, c;
        sincosf(th, &s, &c);
        ps.R[0] = c; ps.R[1] = -s; ps.R[2] = s; ps.R[3] = c;
        ps.dR[0] = -s; ps.dR[1] = -c; ps.dR[2] = c; ps.dR[3] = -s;
        ps.q[2] = th;
    } else {
        const float ph = xa[0], th = xa[1], psi = xa[2];
        float sf, cf, st, ct, sp, cp;
        sincosf(ph, &sf, &cf);
        sincosf(th, &st, &ct);
        sincosf(psi, &sp, &cp);
        float* R = ps.R;
        R[0] = cp * ct; R[1] = cp * st * sf - sp * cf; R[2] = cp * st * cf + sp * sf;
        R[3] = sp * ct; R[4] = sp * st * sf + cp * cf; R[5] = sp * st * cf - cp * sf;
        R[6] = -st;     R[7] = ct * sf;                R[8] = ct * cf;
        float* D = ps.dR;   // d/dphi
        D[0] = 0.f; D[1] = cp * st * cf + sp * sf; D[2] = -cp * st * sf + sp * cf;
        D[3] = 0.f; D[4] = sp * st * cf - cp * sf; D[5] = -sp * st * sf - cp * cf;
        D[6] = 0.f; D[7] = ct * cf;                D[8] = -ct * sf;
        D += 9;             // d/dtheta
        D[0] = -cp * st; D[1] = cp * ct * sf; D[2] = cp * ct * cf;
        D[3] = -sp * st; D[4] = sp * ct * sf; D[5] = sp * ct * cf;
        D[6] = -ct;      D[7] = -st * sf;     D[8] = -st * cf;
        D += 9;             // d/dpsi
        D[0] = -sp * ct; D[1] = -sp * st * sf - cp * cf; D[2] = -sp * st * cf + cp * sf;
        D[3] = cp * ct;  D[4] = cp * st * sf - sp * cf;  D[5] = cp * st * cf + sp * sf;
        D[6] = 0.f;      D[7] = 0.f;                     D[8] = 0.f;
        ps.q[3] = ph; ps.q[4] = th; ps.q[5] = psi;
    }
    // the part centre rho(s) + R(s) o_i; its FP64 copy takes R o_i from FP64
    // trigonometry (only parts with an offset need it)
    double ro64[DIM] = {};
    bool off = false;
#pragma unroll
    for (int c = 0; c < DIM; ++c) off |= o[c] != 0.f;
    if (off) {
        if constexpr (DIM == 2) {
            double s, c;
            sincos((double)xa[0], &s, &c);
            ro64[0] = c * o[0] - s * o[1];
            ro64[1] = s * o[0] + c * o[1];
        } else {
            double sf, cf, st, ct, sp, cp;
            sincos((double)xa[0], &sf, &cf);
            sincos((double)xa[1], &st, &ct);
            sincos((double)xa[2], &sp, &cp);
            const double R64[9] = {cp * ct, cp * st * sf - sp * cf, cp * st * cf + sp * sf,
                                   sp * ct, sp * st * sf + cp * cf, sp * st * cf - cp * sf,
                                   -st,     ct * sf,                ct * cf};
#pragma unroll
            for (int r = 0; r < 3; ++r) ro64[r] = R64[r * 3] * o[0] + R64[r * 3 + 1] * o[1] + R64[r * 3 + 2] * o[2];
        }
    }
#pragma unroll
    for (int r = 0; r < DIM; ++r) {
        const float p = xp[r];
        ps.q[r] = p;
        float ro = 0.f;
#pragma unroll
        for (int c = 0; c < DIM; ++c) ro += ps.R[r * DIM + c] * o[c];
        ps.pos[r] = p + ro;
        ps.pos64[r] = (double)p + ro64[r];
    }
}

// The state entries of the pose at xs (position, attitude) and the part
// offset, loaded into registers (a kernel can issue these loads early).
template <int DIM>
struct PoseInputs {
    float xp[DIM], xa[Pose<DIM>::NATT], o[3];
};

template <int DIM>
__device__ __forceinline__ void load_pose_state(const DevProblem& P, const float* xs, PoseInputs<DIM>& in)
{
#pragma unroll
    for (int r = 0; r < DIM; ++r) in.xp[r] = xs[P.pos_idx[r]];
#pragma unroll
    for (int a = 0; a < Pose<DIM>::NATT; ++a) in.xa[a] = xs[P.att_idx[a]];
}

template <int DIM>
__device__ __forceinline__ void load_pose_offset(const DevProblem& P, int part, PoseInputs<DIM>& in)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) in.o[c] = P.part_off[part * 3 + c];
}

// R(s), dR and the part centre of part `part` at the state xs
template <int DIM>
__device__ __forceinline__ void make_pose(const DevProblem& P, const float* xs, int part, Pose<DIM>& ps)
{
    PoseInputs<DIM> in;
    load_pose_state<DIM>(P, xs, in);
    load_pose_offset<DIM>(P, part, in);
    make_pose_v<DIM>(in.xp, in.xa, in.o, ps);
}

}  // namespace cadmm
