// lbm_adjoint.hpp -- gfx950 kernels of the hand-written adjoint of one step.
//
// Forward step n (arXiv:1703.04594 section 3; order of section 5):
//   g = bc(propagate(f_n)),   f_{n+1} = g + (f^eq(M(g)) - g) / tau,
// M(g) = (rho, j, E) the raw moments of eq. (2).  Given lambda = dL/df_{n+1}:
//
//  collide^T (site-local, rank-4 update):
//    mu_l = (1 - 1/tau) lambda_l + q_rho + q_jx xi_x,l + q_jy xi_y,l + q_E |xi_l|^2
//    with q = J_M^T J_eq^T (lambda / tau): the 4 dot products of lambda with
//    d f^eq / d(rho, u*, T*) pulled back through u = j / rho,
//    T = (E / rho - |u|^2) / 2 and the gravity shift.
//  d step / d tau:  -(1/tau^2) <lambda, f^eq - g> + <lambda / tau, d f^eq / d tau>
//    (the last term through u* = u + tau g, T* = T + tau (1 - tau) g^2 / 2).
//  propagate^T: the pull g_l(s) = f_l(s - e_l) transposes to a push:
//    lambda_n,l(s - e_l) = mu_l(s).  Pushes whose target lies outside the
//    lattice in y belong to wall slots; they land in the ghost rows of the
//    lambda buffer.
//  bc^T: a wall slot (l, s) carries E^w_l rho(m) with rho(m) = sum_k f_k(m) at
//    the mirror site m, so every population of m receives E^w_l mu_l(s); the
//    ghost row value at m's column is exactly that mu_l(s).  Interior slots
//    that no site pushes to (their hop leaves through the wall) get 0.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

struct AdjArgs { double tau, omega, gy; };

// mu <- collide^T lambda at one site, in place; returns the site's d/dtau term.
__device__ __forceinline__ double adjoint_site(const double (&gv)[NPOP], double (&lam)[NPOP], const AdjArgs& a)
{
    using K = ShellK<double>;
    double m0, sx, sy, s2;
    hop_moments<double>(gv, m0, sx, sy, s2);
    const double rho = m0, inv = 1.0 / rho;
    const double ux = C * sx * inv, uy = C * sy * inv;
    const double E = C2 * s2;
    const double T = 0.5 * (E * inv - (ux * ux + uy * uy));
    const double uys = uy + a.tau * a.gy;
    const double th = T - 1.0 + a.tau * (1.0 - a.tau) * a.gy * a.gy * 0.5;
    const double u2 = ux * ux + uys * uys;
    const double cux = C * ux, cuy = C * uys;
    double A0m1[NSHELL], A1[NSHELL], A2[NSHELL], dA0du2[NSHELL], dA0dth[NSHELL];
#pragma unroll
    for (int s = 0; s < NSHELL; ++s) {
        A0m1[s] = u2 * (-0.5 + 0.125 * u2) + th * (K::k1(s) + u2 * K::k2(s) + th * K::k3(s));
        A1[s] = 1.0 - 0.5 * u2 + th * K::k4(s);
        A2[s] = 0.5 - 0.25 * u2 + th * K::k5(s);
        dA0du2[s] = -0.5 + 0.25 * u2 + th * K::k2(s);
        dA0dth[s] = K::k1(s) + u2 * K::k2(s) + 2.0 * th * K::k3(s);
    }
    double SP = 0.0, Sax = 0.0, Say = 0.0, Su2 = 0.0, Sth = 0.0, D = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int s = SHELL[l];
        double P, dPdu2, dPdth;
        const double lw = lam[l] * W_SHELL[s];
        if (l == 0) {
            P = 1.0 + A0m1[0];
            dPdu2 = dA0du2[0];
            dPdth = dA0dth[0];
        } else {
            const double av = hop_dot<double>(l, cux, cuy);
            double t = av * (1.0 / 24.0) + 1.0 / 6.0;
            t = t * av + A2[s];
            t = t * av + A1[s];
            P = 1.0 + (t * av + A0m1[s]);
            const double dPda = A1[s] + av * (2.0 * A2[s] + av * (0.5 + av * (1.0 / 6.0)));
            dPdu2 = dA0du2[s] + av * (-0.5 - 0.25 * av);
            dPdth = dA0dth[s] + av * (K::k4(s) + av * K::k5(s));
            const double Z = lw * dPda;
            if (EX[l] != 0) Sax += (double)EX[l] * Z;
            if (EY[l] != 0) Say += (double)EY[l] * Z;
        }
        SP += lw * P;
        Su2 += lw * dPdu2;
        Sth += lw * dPdth;
        D += lam[l] * (W_SHELL[s] * rho * P - gv[l]);
    }
    const double om = a.omega;
    const double bux = om * rho * (C * Sax + 2.0 * ux * Su2);
    const double buy = om * rho * (C * Say + 2.0 * uys * Su2);
    const double bth = om * rho * Sth;
    const double bP = om * SP;
    const double dtau = -om * om * D + buy * a.gy + bth * (1.0 - 2.0 * a.tau) * a.gy * a.gy * 0.5;
    const double buxt = bux - bth * ux, buyt = buy - bth * uy;
    const double bE = 0.5 * bth * inv;
    const double bjx = buxt * inv, bjy = buyt * inv;
    const double brho = bP - (buxt * ux + buyt * uy) * inv - 0.5 * bth * E * inv * inv;
    const double cjx = C * bjx, cjy = C * bjy, c2E = C2 * bE;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        double mu = (1.0 - om) * lam[l] + brho;
        if (EX[l] != 0) mu += (double)EX[l] * cjx;
        if (EY[l] != 0) mu += (double)EY[l] * cjy;
        if (R2_OF(l) != 0) mu += (double)R2_OF(l) * c2E;
        lam[l] = mu;
    }
    return dtau;
}

// One block sum of a double into partials[blockIdx linear].
__device__ __forceinline__ void block_sum1(double v, double* __restrict__ partials)
{
    double a[1] = {v};
    block_sum_store<1>(a, partials + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

template <typename S, bool WALLS>
__global__ __launch_bounds__(SITE_THREADS) void k_adj_collide_push(
    const S* __restrict__ fn, Geo g, const double* __restrict__ lam_in, double* __restrict__ lam_out, Geo lg,
    AdjArgs a, const double* __restrict__ wall_rho, WallTable wt, double* __restrict__ partials)
{
    const int x = blockIdx.y;
    const int y = blockIdx.x * SITE_THREADS + threadIdx.x;
    double dtau = 0.0;
    if (y < g.ly) {
        double gv[NPOP], lam[NPOP];
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            const int xs = wrap_x(x - EX[l], g.lx);
            int ys = y - EY[l];
            if (!WALLS) ys = ys < 0 ? ys + g.ly : (ys >= g.ly ? ys - g.ly : ys);
            double v = (double)fn[(size_t)l * g.plane + g.origin + (long long)xs * g.lyp + ys];
            if (Store<S>::shifted) v += wt.w[l];
            gv[l] = v;
        }
        if (WALLS && (y < 3 || y >= g.ly - 3)) {
#pragma unroll
            for (int l = 0; l < NPOP; ++l) {
                if (EY[l] == 0) continue;
                const int wall = EY[l] > 0 ? 0 : 1;
                const int r = wall == 0 ? y : g.ly - 1 - y;
                const int en = wall == 0 ? EY[l] : -EY[l];
                if (en > r) {
                    const int xs = wrap_x(x - EX[l], g.lx);
                    gv[l] = wt.ew[wall][l] * wall_rho[(wall * 3 + (en - r - 1)) * g.lx + xs];
                }
            }
        }
        const double* lp = lam_in + lg.origin + (long long)x * lg.lyp + y;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) lam[l] = lp[(size_t)l * lg.plane];
        dtau = adjoint_site(gv, lam, a);
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            const int xd = wrap_x(x - EX[l], g.lx);
            int yd = y - EY[l];
            if (!WALLS) yd = yd < 0 ? yd + g.ly : (yd >= g.ly ? yd - g.ly : yd);
            lam_out[(size_t)l * lg.plane + lg.origin + (long long)xd * lg.lyp + yd] = lam[l];
        }
    }
    block_sum1(dtau, partials);
}

// bc^T and the zeroing of slots nobody pushes to: thread per (wall, row, x).
__global__ __launch_bounds__(256) void k_adj_bc_fix(double* __restrict__ lam, Geo lg, WallTable wt)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= 6 * lg.lx) return;
    const int x = t % lg.lx, wr = t / lg.lx;
    const int wall = wr / 3, r = wr % 3;
    const int y = wall == 0 ? r : lg.ly - 1 - r;
    const int yg = wall == 0 ? -r - 1 : lg.ly + r;
    double* col = lam + lg.origin + (long long)x * lg.lyp;
    double beta = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int en = wall == 0 ? EY[l] : -EY[l];
        if (en >= r + 1) beta += wt.ew[wall][l] * col[(size_t)l * lg.plane + yg];
    }
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int en = wall == 0 ? EY[l] : -EY[l];
        double* p = col + (size_t)l * lg.plane + y;
        const double v = (-en > r) ? 0.0 : *p;
        *p = v + beta;
    }
}

// lambda_l = d(x,y) dT/df_l = d (|xi_l - u|^2 - 2T) / (2 rho), with
// d = dT(x,y) (SEED) or d = T - T_target (LOSS, plus 1/2 d^2 into partials).
template <typename S, bool LOSS>
__global__ __launch_bounds__(SITE_THREADS) void k_adj_seed_T(const S* __restrict__ fbuf, Geo g, double* __restrict__ lam, Geo lg,
                                                          const double* __restrict__ d_in, double* __restrict__ partials)
{
    const int x = blockIdx.y;
    const int y = blockIdx.x * SITE_THREADS + threadIdx.x;
    double loss = 0.0;
    if (y < g.ly) {
        double rho, ux, uy, T;
        site_macros<S>(fbuf + g.origin + (long long)x * g.lyp + y, g.plane, rho, ux, uy, T);
        double d = d_in[(long long)x * g.ly + y];
        if (LOSS) { d = T - d; loss = 0.5 * d * d; }
        const double k = d / (2.0 * rho);
        double* lp = lam + lg.origin + (long long)x * lg.lyp + y;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            const double dx = C * EX[l] - ux, dy = C * EY[l] - uy;
            lp[(size_t)l * lg.plane] = k * (dx * dx + dy * dy - 2.0 * T);
        }
    }
    if (LOSS) block_sum1(loss, partials);
}

// dL/dP from lambda_0 for f_0 = f^eq(rho0(P), 0, T0(P)):
//   T0 = t_mid - t_amp tanh(z), z = (y - y_mid - P) / width, rho0 = p0 / T0,
//   f^eq_l(rho, 0, T) = w_l rho (1 + th K1 + th^2 K3), th = T - 1.
__global__ __launch_bounds__(SITE_THREADS) void k_adj_init_rt(const double* __restrict__ lam, Geo lg, const double* __restrict__ P,
                                                           RtProfile pr, double* __restrict__ dP)
{
    using K = ShellK<double>;
    const int x = blockIdx.y;
    const int y = blockIdx.x * SITE_THREADS + threadIdx.x;
    if (y >= lg.ly) return;
    const long long s = (long long)x * lg.ly + y;
    const double th_z = tanh((y - pr.y_mid - P[s]) / pr.width);
    const double T0 = pr.t_mid - pr.t_amp * th_z;
    const double r0 = pr.p0 / T0;
    const double dT = pr.t_amp * (1.0 - th_z * th_z) / pr.width;
    const double dr = -pr.p0 / (T0 * T0) * dT;
    const double th = T0 - 1.0;
    const double* lp = lam + lg.origin + (long long)x * lg.lyp + y;
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int sh = SHELL[l];
        const double Pl = 1.0 + th * (K::k1(sh) + th * K::k3(sh));
        const double dPl = K::k1(sh) + 2.0 * th * K::k3(sh);
        acc += lp[(size_t)l * lg.plane] * W_SHELL[sh] * (Pl * dr + r0 * dPl * dT);
    }
    dP[s] = acc;
}

}  // namespace lbm
