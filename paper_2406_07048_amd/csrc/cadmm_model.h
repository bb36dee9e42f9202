// Nonlinear dynamics s_{t+1} = s_t + dt f_c(s_t, u_t) (Sec. IV-A eq.
// system_eqn) of the built-in models, written once for the host (FP64, the
// closed-loop plant) and the device (FP64 values with one forward-mode
// tangent, the SQP linearisation).
//   model 1 (kinematic bicycle, s = (p_x, p_y, theta, v), u = (a, delta),
//     par = (dt, wheelbase L)): f_c = (v cos theta, v sin theta, v tan(delta) / L, a);
//   model 2 (quadrotor, s = (p, v, phi theta psi, body rates w), u = (dF, tau),
//     par = (dt, m, J_x, J_y, J_z, g)): p' = v, v' = (g + dF / m) R e_3 - g e_3
//     with R = R_z(psi) R_y(theta) R_x(phi), the ZYX Euler-angle rates of the
//     body rates, and Euler's equations J w' = tau + (J w) x w for a diagonal J.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace cadmm {

// a value and one tangent
struct Tan {
    double v, d;
};
__host__ __device__ inline Tan operator+(Tan a, Tan b) { return {a.v + b.v, a.d + b.d}; }
__host__ __device__ inline Tan operator-(Tan a, Tan b) { return {a.v - b.v, a.d - b.d}; }
__host__ __device__ inline Tan operator*(Tan a, Tan b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__host__ __device__ inline Tan operator*(double a, Tan b) { return {a * b.v, a * b.d}; }
__host__ __device__ inline Tan operator/(Tan a, Tan b)
{
    const double q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
__host__ __device__ inline Tan operator/(Tan a, double b) { return {a.v / b, a.d / b}; }
__host__ __device__ inline Tan tsin(Tan a) { return {sin(a.v), cos(a.v) * a.d}; }
__host__ __device__ inline Tan tcos(Tan a) { return {cos(a.v), -sin(a.v) * a.d}; }
__host__ __device__ inline Tan ttan(Tan a)
{
    const double t = tan(a.v);
    return {t, (1.0 + t * t) * a.d};
}
__host__ __device__ inline double tsin(double a) { return sin(a); }
__host__ __device__ inline double tcos(double a) { return cos(a); }
__host__ __device__ inline double ttan(double a) { return tan(a); }
// the same with the sine, cosine or tangent of the argument's value given
// (formed once per state and shared by the forward-mode columns)
__host__ __device__ inline Tan tsin_of(Tan a, double sv, double cv) { return {sv, cv * a.d}; }
__host__ __device__ inline Tan tcos_of(Tan a, double sv, double cv) { return {cv, -sv * a.d}; }
__host__ __device__ inline Tan ttan_of(Tan a, double tv) { return {tv, (1.0 + tv * tv) * a.d}; }
__host__ __device__ inline double tsin_of(double, double sv, double) { return sv; }
__host__ __device__ inline double tcos_of(double, double, double cv) { return cv; }
__host__ __device__ inline double ttan_of(double, double tv) { return tv; }
template <class T> __host__ __device__ inline T constant(double c);
template <> __host__ __device__ inline Tan constant<Tan>(double c) { return Tan{c, 0.0}; }
template <> __host__ __device__ inline double constant<double>(double c) { return c; }

inline constexpr int model_ns(int model) { return model == 1 ? 4 : 12; }
inline constexpr int model_nu(int model) { return model == 1 ? 2 : 4; }

// Sines and cosines of the angles of a state and input (model 1: theta,
// and tan(delta); model 2: phi, theta, psi), in FP64.
struct ModelTrig {
    double s[3], c[3], tn;
};
template <class V>
__host__ __device__ inline void model_trig(int model, const V* s, const V* u, ModelTrig& tr)
{
    if (model == 1) {
        tr.s[0] = sin((double)s[2]);
        tr.c[0] = cos((double)s[2]);
        tr.tn = tan((double)u[1]);
    } else {
        for (int k = 0; k < 3; ++k) {
            tr.s[k] = sin((double)s[6 + k]);
            tr.c[k] = cos((double)s[6 + k]);
        }
    }
}

// f_c(S, U) of model 1 or 2 into f (n_s entries); with tr the sines and
// cosines of the angles are taken from it (the same values)
template <class T>
__host__ __device__ inline void model_fc(int model, const double* par, const T* S, const T* U, T* f,
                                         const ModelTrig* tr = nullptr)
{
    auto SIN = [&](const T& a, int k) { return tr ? tsin_of(a, tr->s[k], tr->c[k]) : tsin(a); };
    auto COS = [&](const T& a, int k) { return tr ? tcos_of(a, tr->s[k], tr->c[k]) : tcos(a); };
    if (model == 1) {
        f[0] = S[3] * COS(S[2], 0);
        f[1] = S[3] * SIN(S[2], 0);
        f[2] = S[3] * (tr ? ttan_of(U[1], tr->tn) : ttan(U[1])) / par[1];
        f[3] = U[0];
    } else {
        const double m = par[1], Jx = par[2], Jy = par[3], Jz = par[4], g = par[5];
        const T cph = COS(S[6], 0), sph = SIN(S[6], 0), cth = COS(S[7], 1), sth = SIN(S[7], 1);
        const T cps = COS(S[8], 2), sps = SIN(S[8], 2);
        const T acc = constant<T>(g) + U[0] / m;
        f[0] = S[3]; f[1] = S[4]; f[2] = S[5];
        f[3] = acc * (cps * sth * cph + sps * sph);
        f[4] = acc * (sps * sth * cph - cps * sph);
        f[5] = acc * (cth * cph) - constant<T>(g);
        const T p = S[9], q = S[10], r = S[11];
        const T qr = q * sph + r * cph;
        f[6] = p + qr * sth / cth;
        f[7] = q * cph - r * sph;
        f[8] = qr / cth;
        f[9] = (U[1] + (Jy - Jz) * (q * r)) / Jx;
        f[10] = (U[2] + (Jz - Jx) * (r * p)) / Jy;
        f[11] = (U[3] + (Jx - Jy) * (p * q)) / Jz;
    }
}

}  // namespace cadmm
