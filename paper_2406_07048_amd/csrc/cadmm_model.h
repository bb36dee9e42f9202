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
template <class T> __host__ __device__ inline T constant(double c);
template <> __host__ __device__ inline Tan constant<Tan>(double c) { return Tan{c, 0.0}; }
template <> __host__ __device__ inline double constant<double>(double c) { return c; }

inline constexpr int model_ns(int model) { return model == 1 ? 4 : 12; }
inline constexpr int model_nu(int model) { return model == 1 ? 2 : 4; }

// f_c(S, U) of model 1 or 2 into f (n_s entries)
template <class T>
__host__ __device__ inline void model_fc(int model, const double* par, const T* S, const T* U, T* f)
{
    if (model == 1) {
        f[0] = S[3] * tcos(S[2]);
        f[1] = S[3] * tsin(S[2]);
        f[2] = S[3] * ttan(U[1]) / par[1];
        f[3] = U[0];
    } else {
        const double m = par[1], Jx = par[2], Jy = par[3], Jz = par[4], g = par[5];
        const T cph = tcos(S[6]), sph = tsin(S[6]), cth = tcos(S[7]), sth = tsin(S[7]);
        const T cps = tcos(S[8]), sps = tsin(S[8]);
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
