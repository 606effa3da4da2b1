// lbm_site.hpp -- per-site arithmetic of the D2Q37 step on gfx950.
//
// arXiv:1703.04594, section 3: moments of eq. (2), BGK relaxation of
// eq. (1) towards the 4th-order Hermite equilibrium, with gravity entering as
// a shift of the equilibrium's velocity and temperature.  Two storage forms:
//  - absolute:  f_l, computed in FP64;
//  - shifted:   d_l = f_l - w_l (deviation from the rest state rho = 1, u = 0,
//               T = 1, whose equilibrium is w_l), computed in FP32.  All sums
//               are of deviations, so their rounding error scales with the
//               departure from rest, not with the populations themselves.
//
// The equilibrium is evaluated per site in Horner form in a = xi_l . u:
//   f^eq_l = w_l rho (A0 + a (A1 + a (A2 + a (1/6 + a/24))))
// with shell coefficients (x2 = |xi|^2, th = T - 1, u2 = |u|^2)
//   A0 = 1 - u2/2 + u2^2/8 + th ((x2-2)/2 + u2 (4-x2)/4 + th (x2^2-8x2+8)/8)
//   A1 = 1 - u2/2 + th (x2-4)/2
//   A2 = 1/2 - u2/4 + th (x2-6)/4
// which is the expanded 4th-order Hermite expansion regrouped by powers of a.
#pragma once

#include <hip/hip_runtime.h>

#include "d2q37_tables.h"

namespace lbm {

using namespace d2q37;

constexpr int R2_OF(int l) { return EX[l] * EX[l] + EY[l] * EY[l]; }

// |xi_l|^2 in FP64 as the moments define it: the hop xi_l = c e_l rounded per
// component, then squared and summed.  The FP64 step takes the equilibrium's
// shell constants and the temperature's second moment from these values.
// With c^2 |e|^2 rounded once instead (a different rounding of the same
// constant), the FP64 temperature is biased by ~1e-16 relative at every
// step; energy is conserved, so the bias accumulates, and the state drifts
// from one computed with the per-component rounding by ~1.5e-15 per step.
// Both arrays are constant-evaluated, so every operation rounds once.
constexpr double xi2_of_pop(int l)
{
    const double xx = C * EX[l], yy = C * EY[l];
    return xx * xx + yy * yy;
}
constexpr double xi2_of_shell(int s)
{
    for (int l = 0; l < NPOP; ++l)
        if (SHELL[l] == s) return xi2_of_pop(l);
    return 0.0;
}
struct Xi2Tables {
    double pop[NPOP];
    double shell[NSHELL];
    double k1[NSHELL], k2[NSHELL], k3[NSHELL], k4[NSHELL], k5[NSHELL];
};
constexpr Xi2Tables make_xi2_tables()
{
    Xi2Tables t{};
    for (int l = 0; l < NPOP; ++l) t.pop[l] = xi2_of_pop(l);
    for (int s = 0; s < NSHELL; ++s) {
        const double x2 = xi2_of_shell(s);
        t.shell[s] = x2;
        t.k1[s] = (x2 - 2.0) / 2.0;
        t.k2[s] = (4.0 - x2) / 4.0;
        t.k3[s] = (x2 * x2 - 8.0 * x2 + 8.0) / 8.0;
        t.k4[s] = (x2 - 4.0) / 2.0;
        t.k5[s] = (x2 - 6.0) / 4.0;
    }
    return t;
}
constexpr Xi2Tables XI2 = make_xi2_tables();

// Shell constants of the Hermite coefficients, evaluated at compile time:
// FP64 from the tables above, FP32 from c^2 |e|^2 in FP32.
template <typename C> struct ShellK;
template <> struct ShellK<double> {
    static constexpr double x2(int s) { return XI2.shell[s]; }
    static constexpr double k1(int s) { return XI2.k1[s]; }
    static constexpr double k2(int s) { return XI2.k2[s]; }
    static constexpr double k3(int s) { return XI2.k3[s]; }
    static constexpr double k4(int s) { return XI2.k4[s]; }
    static constexpr double k5(int s) { return XI2.k5[s]; }
};
template <> struct ShellK<float> {
    using F = float;
    static constexpr F x2(int s) { return F(SHELL_R2[s]) * F(C2); }
    static constexpr F k1(int s) { return (F(C2) * F(SHELL_R2[s]) - F(2)) / F(2); }
    static constexpr F k2(int s) { return (F(4) - F(C2) * F(SHELL_R2[s])) / F(4); }
    static constexpr F k3(int s) {
        return (F(C2) * F(SHELL_R2[s]) * F(C2) * F(SHELL_R2[s]) - F(8) * F(C2) * F(SHELL_R2[s]) + F(8)) / F(8);
    }
    static constexpr F k4(int s) { return (F(C2) * F(SHELL_R2[s]) - F(4)) / F(2); }
    static constexpr F k5(int s) { return (F(C2) * F(SHELL_R2[s]) - F(6)) / F(4); }
};

// FP64 second moment sum_l |xi_l|^2 f_l with the per-population |xi_l|^2.
template <typename V>
__device__ __forceinline__ double xi2_moment(const V (&f)[NPOP])
{
    double e = 0.0;
#pragma unroll
    for (int l = 1; l < NPOP; ++l) e += XI2.pop[l] * (double)f[l];
    return e;
}

template <typename C> __device__ __host__ constexpr C wshell(int s);
template <> __device__ __host__ constexpr double wshell<double>(int s) { return W_SHELL[s]; }
template <> __device__ __host__ constexpr float wshell<float>(int s) { return W_SHELL_F[s]; }
template <typename C> __device__ __host__ constexpr C cscale();
template <> __device__ __host__ constexpr double cscale<double>() { return C; }
template <> __device__ __host__ constexpr float cscale<float>() { return C_F; }
template <typename C> __device__ __host__ constexpr C c2scale();
template <> __device__ __host__ constexpr double c2scale<double>() { return C2; }
template <> __device__ __host__ constexpr float c2scale<float>() { return C2_F; }

// Integer-hop moments: m0 = sum f, sx = sum ex f, sy = sum ey f,
// s2 = sum |e|^2 f.  Zero hop components are skipped at compile time.
template <typename C>
__device__ __forceinline__ void hop_moments(const C (&f)[NPOP], C& m0, C& sx, C& sy, C& s2)
{
    m0 = C(0); sx = C(0); sy = C(0); s2 = C(0);
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        m0 += f[l];
        if (EX[l] != 0) sx += C(EX[l]) * f[l];
        if (EY[l] != 0) sy += C(EY[l]) * f[l];
        if (R2_OF(l) != 0) s2 += C(R2_OF(l)) * f[l];
    }
}

// The same moments of FP32 populations, accumulated in FP64.
__device__ __forceinline__ void hop_moments_wide(const float (&f)[NPOP], double& m0, double& sx, double& sy, double& s2)
{
    m0 = 0.0; sx = 0.0; sy = 0.0; s2 = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const double v = (double)f[l];
        m0 += v;
        if (EX[l] != 0) sx += (double)EX[l] * v;
        if (EY[l] != 0) sy += (double)EY[l] * v;
        if (R2_OF(l) != 0) s2 += (double)R2_OF(l) * v;
    }
}

template <typename C>
__host__ __device__ __forceinline__ C hop_dot(int l, C cux, C cuy)
{
    C a = C(0);
    if (EX[l] != 0 && EY[l] != 0) a = C(EX[l]) * cux + C(EY[l]) * cuy;
    else if (EX[l] != 0) a = C(EX[l]) * cux;
    else if (EY[l] != 0) a = C(EY[l]) * cuy;
    return a;
}

struct CollideArgs {
    double omega;    // 1 / tau
    double tau_g;    // tau * g_y   (velocity shift)
    double grav_th;  // tau (1 - tau) g_y^2 / 2   (temperature shift)
    double g;        // g_y
    float omega_f, tau_g_f, grav_th_f, g_f;
};

template <typename C> __device__ __forceinline__ C arg_omega(const CollideArgs& a);
template <> __device__ __forceinline__ double arg_omega<double>(const CollideArgs& a) { return a.omega; }
template <> __device__ __forceinline__ float arg_omega<float>(const CollideArgs& a) { return a.omega_f; }
template <typename C> __device__ __forceinline__ C arg_taug(const CollideArgs& a);
template <> __device__ __forceinline__ double arg_taug<double>(const CollideArgs& a) { return a.tau_g; }
template <> __device__ __forceinline__ float arg_taug<float>(const CollideArgs& a) { return a.tau_g_f; }
template <typename C> __device__ __forceinline__ C arg_gth(const CollideArgs& a);
template <> __device__ __forceinline__ double arg_gth<double>(const CollideArgs& a) { return a.grav_th; }
template <> __device__ __forceinline__ float arg_gth<float>(const CollideArgs& a) { return a.grav_th_f; }
template <typename C> __device__ __forceinline__ C arg_g(const CollideArgs& a);
template <> __device__ __forceinline__ double arg_g<double>(const CollideArgs& a) { return a.g; }
template <> __device__ __forceinline__ float arg_g<float>(const CollideArgs& a) { return a.g_f; }

// BGK collision of one site, in place.  SHIFTED: f holds deviations d_l.
//
// In the shifted (FP32) form the relaxed populations are finally projected
// back onto the exact post-collision moments.  In exact arithmetic the
// equilibrium has the moments of f (mass, momentum plus tau*rho*g, energy
// plus the work of the gravity shift), so the projection is zero; in FP32 the
// rounded weights and scale break those identities by ~1e-8 per step, which
// would otherwise drift mass and energy systematically.  The moment sums on
// both sides of the projection are accumulated in FP64: an FP32 sum of 37
// terms is off by ~1e-8, and at a site whose state changes slowly that error
// repeats with the same sign step after step, so it would bias the conserved
// moments just as the rounded weights do.  The correction is
// w_l (a + b ex + c ey + d |e|^2); its Gram matrix sum_l w_l v v^T with
// v = (1, ex, ey, |e|^2) is fixed by the quadrature (sum w = 1,
// sum w ex^2 = 1/c^2, sum w |e|^2 = 2/c^2, sum w |e|^4 = 8/c^4), which gives
// a = 2 d0 - (c^2/2) d2, b = c^2 dx, c' = c^2 dy, d = -(c^2/2) d0 + (c^4/4) d2
// for the moment defects (d0, dx, dy, d2).
//
// WIDE = false (shifted form only) keeps every sum in FP32 as well: the
// same collision with FP32 moment sums on both sides of the projection, for
// measuring what the FP64 sums buy.
template <typename C, bool SHIFTED, bool WIDE = true>
__device__ __forceinline__ void collide_site(C (&f)[NPOP], const CollideArgs& args)
{
    using K = ShellK<C>;
    const C omega = arg_omega<C>(args);
    C m0, sx, sy, s2;
    double m0d = 0.0, sxd = 0.0, syd = 0.0, s2d = 0.0;   // FP64 sums (shifted form)
    if constexpr (SHIFTED && WIDE) {
        hop_moments_wide(f, m0d, sxd, syd, s2d);
        m0 = (C)m0d; sx = (C)sxd; sy = (C)syd; s2 = (C)s2d;
    } else if constexpr (SHIFTED) {
        hop_moments<C>(f, m0, sx, sy, s2);
    } else {
        hop_moments<C>(f, m0, sx, sy, s2);
    }
    const C rho = SHIFTED ? C(1) + m0 : m0;
    const C inv = C(1) / rho;
    const C ux = cscale<C>() * sx * inv;
    const C uy0 = cscale<C>() * sy * inv;   // velocity of f, before the gravity shift
    C th;
    if constexpr (SHIFTED) {
        // T - 1 = (sum (x2 - 2) d) / (2 rho) - u2 / 2
        th = (c2scale<C>() * s2 - C(2) * m0) * inv * C(0.5) - (ux * ux + uy0 * uy0) * C(0.5);
    } else {
        static_assert(sizeof(C) == 8, "the absolute form is FP64");
        th = (xi2_moment(f) * inv - (ux * ux + uy0 * uy0)) * C(0.5) - C(1);
    }
    const C uy = uy0 + arg_taug<C>(args);
    th += arg_gth<C>(args);
    const C u2 = ux * ux + uy * uy;
    const C cux = cscale<C>() * ux, cuy = cscale<C>() * uy;
    // shell-independent parts
    const C b1 = C(1) - C(0.5) * u2;             // A1 without th
    const C b2 = C(0.5) - C(0.25) * u2;          // A2 without th
    const C b0m1 = u2 * (C(-0.5) + C(0.125) * u2); // A0 - 1 without th
    // populations are ordered by shell: form each shell's coefficients just
    // before its populations, so only one shell's worth is live
#pragma unroll
    for (int s = 0; s < NSHELL; ++s) {
        const C A0m1 = b0m1 + th * (K::k1(s) + u2 * K::k2(s) + th * K::k3(s));
        const C A1 = b1 + th * K::k4(s);
        const C A2 = b2 + th * K::k5(s);
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            if (SHELL[l] != s) continue;
            C pm;   // P - 1 = A0 - 1 + a (A1 + a (A2 + a (1/6 + a/24)))
            if (l == 0) {
                pm = A0m1;
            } else {
                const C a = hop_dot<C>(l, cux, cuy);
                C t = a * C(1.0 / 24.0) + C(1.0 / 6.0);
                t = t * a + A2;
                t = t * a + A1;
                pm = t * a + A0m1;
            }
            C feq;
            if constexpr (SHIFTED) {
                // d^eq = w ((rho - 1) P + (P - 1)) = w (m0 + rho (P - 1))
                feq = wshell<C>(s) * (m0 + rho * pm);
            } else {
                feq = wshell<C>(s) * rho * (C(1) + pm);
            }
            f[l] = f[l] + omega * (feq - f[l]);
        }
    }
    if constexpr (SHIFTED) {
        const C g = arg_g<C>(args);
        const C c2 = c2scale<C>();
        C d0, dx, dy, d2;
        if constexpr (WIDE) {
            double M0, MX, MY, M2;
            hop_moments_wide(f, M0, MX, MY, M2);
            d0 = (C)(m0d - M0);
            dx = (C)(sxd - MX);
            dy = (C)(syd + (1.0 + m0d) * (args.g / cscale<double>()) - MY);
            d2 = (C)(s2d + (double)(rho * (C(2) * g * uy0 + g * g) / c2) - M2);
        } else {
            C M0, MX, MY, M2;
            hop_moments<C>(f, M0, MX, MY, M2);
            d0 = m0 - M0;
            dx = sx - MX;
            dy = sy + rho * (g / cscale<C>()) - MY;
            d2 = s2 + rho * (C(2) * g * uy0 + g * g) / c2 - M2;
        }
        const C ka = C(2) * d0 - C(0.5) * c2 * d2;
        const C kb = c2 * dx, kc = c2 * dy;
        const C kd = C(-0.5) * c2 * d0 + C(0.25) * c2 * c2 * d2;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            C corr = ka;
            if (EX[l] != 0) corr += C(EX[l]) * kb;
            if (EY[l] != 0) corr += C(EY[l]) * kc;
            if (R2_OF(l) != 0) corr += C(R2_OF(l)) * kd;
            f[l] += wshell<C>(SHELL[l]) * corr;
        }
    }
}

// Equilibrium of given fields, FP64 (initial states and wall tables).
// Returns f^eq_l - w_l when SHIFTED, f^eq_l otherwise.
template <bool SHIFTED>
__device__ __host__ __forceinline__ double feq_pop(int l, double rho, double ux, double uy, double T)
{
    using K = ShellK<double>;
    const int s = SHELL[l];
    const double th = T - 1.0;
    const double u2 = ux * ux + uy * uy;
    const double a = C * (EX[l] * ux + EY[l] * uy);
    const double A0m1 = u2 * (-0.5 + 0.125 * u2) + th * (K::k1(s) + u2 * K::k2(s) + th * K::k3(s));
    const double A1 = 1.0 - 0.5 * u2 + th * K::k4(s);
    const double A2 = 0.5 - 0.25 * u2 + th * K::k5(s);
    double t = a * (1.0 / 24.0) + 1.0 / 6.0;
    t = t * a + A2;
    t = t * a + A1;
    const double pm = t * a + A0m1;
    if (SHIFTED) return W_SHELL[s] * ((rho - 1.0) + rho * pm);
    return W_SHELL[s] * rho * (1.0 + pm);
}

}  // namespace lbm
