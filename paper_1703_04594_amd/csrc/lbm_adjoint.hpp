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
//  propagate^T and bc^T, evaluated as a pull by the step that needs lambda_n
//  (the next reverse step, or the readers of lambda): the buffer holds mu at
//  each site, and
//    lambda_n,l(s) = [s + e_l inside the lattice] mu_l(s + e_l) + beta(s),
//  since the pull g_l(s') = f_l(s' - e_l) reads f_l(s) only from s' = s + e_l,
//  and a slot s' whose source s is inside is never a wall slot.  beta (rows
//  0-2 and ly-3..ly-1 only) is bc^T: a wall slot (l, w) carries
//  E^w_l rho(m) with rho(m) = sum_k f_k(m) at the mirror site m of its
//  source, so every population of m receives E^w_l mu_l(w).  For a site s
//  in row r from a wall, the wall slots mirroring onto it are
//  w = (x + e_x,l, e_n - 1 - r) counted from that wall, for each l whose
//  component e_n into the lattice exceeds r.
//  Storing mu at its own site keeps every store aligned (a push would write
//  e_y-shifted partial lines) and folds bc^T into the gather.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

struct AdjArgs { double tau, omega, gy; };

// Per-site scalars of collide^T that depend only on the gathered moments.
struct AdjSite {
    double rho, inv, ux, uy, uys, E, th, u2, cux, cuy;
};

__host__ __device__ __forceinline__ AdjSite adj_site_scalars(double m0, double sx, double sy, double s2, const AdjArgs& a)
{
    AdjSite q;
    q.rho = m0;
    q.inv = 1.0 / m0;
    q.ux = C * sx * q.inv;
    q.uy = C * sy * q.inv;
    q.E = C2 * s2;
    const double T = 0.5 * (q.E * q.inv - (q.ux * q.ux + q.uy * q.uy));
    q.uys = q.uy + a.tau * a.gy;
    q.th = T - 1.0 + a.tau * (1.0 - a.tau) * a.gy * a.gy * 0.5;
    q.u2 = q.ux * q.ux + q.uys * q.uys;
    q.cux = C * q.ux;
    q.cuy = C * q.uys;
    return q;
}

// OPP.v[l]: index of the hop opposite to l (e_l' = -e_l; same shell),
// tabulated at compile time so that indexing with an unrolled l folds.
struct OppTable { int v[NPOP]; };
constexpr OppTable make_opp()
{
    OppTable t{};
    for (int l = 0; l < NPOP; ++l)
        for (int k = 0; k < NPOP; ++k)
            if (EX[k] == -EX[l] && EY[k] == -EY[l]) t.v[l] = k;
    return t;
}
constexpr OppTable OPP = make_opp();
static_assert(OPP.v[0] == 0 && OPP.v[1] == 3 && OPP.v[2] == 4 && OPP.v[36] == 32, "opposite hops");

// mu <- collide^T lambda at one site, in place, given the gathered moments
// (m0, sx, sy, s2) and Lg = sum_l lambda_l g_l; returns the site's d/dtau term.
//
// The equilibrium factor of population l is a polynomial in a_l = xi_l . u*,
//   P(a) = 1 + A0m1 + A1 a + A2 a^2 + a^3/6 + a^4/24,
// with shell coefficients A0m1, A1, A2 (functions of |u*|^2 and theta).
// collide^T needs, per shell, sum lambda P, sum e lambda dP/da, and
// sum lambda dP/d|u|^2, sum lambda dP/dtheta.  Opposite hops l, l' share the
// shell and have a_l' = -a_l, so each polynomial splits into an even part
// (shared) and an odd part (sign flipped): a pair contributes through
// lambda_l + lambda_l' and lambda_l - lambda_l' only, and every polynomial is
// evaluated once per pair.  Shell coefficients are formed shell by shell
// (populations are ordered by shell), so only one shell's worth is live.
__host__ __device__ __forceinline__ double adjoint_site(double m0, double sx, double sy, double s2, double Lg,
                                                        double (&lam)[NPOP], const AdjArgs& a)
{
    using K = ShellK<double>;
    const AdjSite q = adj_site_scalars(m0, sx, sy, s2, a);
    double SP = 0.0, Sax = 0.0, Say = 0.0, Su2 = 0.0, Sth = 0.0;
#pragma unroll
    for (int s = 0; s < NSHELL; ++s) {
        const double A0m1 = q.u2 * (-0.5 + 0.125 * q.u2) + q.th * (K::k1(s) + q.u2 * K::k2(s) + q.th * K::k3(s));
        const double A1 = 1.0 - 0.5 * q.u2 + q.th * K::k4(s);
        const double A2 = 0.5 - 0.25 * q.u2 + q.th * K::k5(s);
        const double dA0du2 = -0.5 + 0.25 * q.u2 + q.th * K::k2(s);
        const double dA0dth = K::k1(s) + q.u2 * K::k2(s) + 2.0 * q.th * K::k3(s);
        double sP = 0.0, sax = 0.0, say = 0.0, su2 = 0.0, sth = 0.0;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            if (SHELL[l] != s) continue;
            if (l == 0) {
                sP += lam[0] * (1.0 + A0m1);
                su2 += lam[0] * dA0du2;
                sth += lam[0] * dA0dth;
                continue;
            }
            const int m = OPP.v[l];
            if (m < l) continue;                 // each pair once, from its first hop
            const double av = hop_dot<double>(l, q.cux, q.cuy);
            const double a2 = av * av;
            const double sg = lam[l] + lam[m], dl = lam[l] - lam[m];
            // even and odd parts of P, dP/da, dP/d|u|^2, dP/dtheta
            const double PE = (1.0 + A0m1) + a2 * (A2 + a2 * (1.0 / 24.0));
            const double PO = av * (A1 + a2 * (1.0 / 6.0));
            const double DE = A1 + 0.5 * a2;
            const double DO = av * (2.0 * A2 + a2 * (1.0 / 6.0));
            sP += sg * PE + dl * PO;
            const double Z = dl * DE + sg * DO;   // sum over the pair of sign(e) lambda dP/da
            if (EX[l] != 0) sax += (double)EX[l] * Z;
            if (EY[l] != 0) say += (double)EY[l] * Z;
            su2 += sg * (dA0du2 - 0.25 * a2) - 0.5 * (dl * av);
            sth += sg * (dA0dth + K::k5(s) * a2) + K::k4(s) * (dl * av);
        }
        const double ws = W_SHELL[s];
        SP += ws * sP;
        Sax += ws * sax;
        Say += ws * say;
        Su2 += ws * su2;
        Sth += ws * sth;
    }
    const double om = a.omega;
    const double bux = om * q.rho * (C * Sax + 2.0 * q.ux * Su2);
    const double buy = om * q.rho * (C * Say + 2.0 * q.uys * Su2);
    const double bth = om * q.rho * Sth;
    const double bP = om * SP;
    // sum_l lambda_l (f^eq_l - g_l) = rho SP - Lg
    const double D = q.rho * SP - Lg;
    const double dtau = -om * om * D + buy * a.gy + bth * (1.0 - 2.0 * a.tau) * a.gy * a.gy * 0.5;
    const double buxt = bux - bth * q.ux, buyt = buy - bth * q.uy;
    const double bE = 0.5 * bth * q.inv;
    const double bjx = buxt * q.inv, bjy = buyt * q.inv;
    const double brho = bP - (buxt * q.ux + buyt * q.uy) * q.inv - 0.5 * bth * q.E * q.inv * q.inv;
    const double cjx = C * bjx, cjy = C * bjy, c2E = C2 * bE;
    // mu_l = (1 - 1/tau) lambda_l + brho + xi_l . bj + |xi_l|^2 bE: the |e|^2
    // part is shared by a pair, the e part flips sign
    lam[0] = (1.0 - om) * lam[0] + brho;
#pragma unroll
    for (int l = 1; l < NPOP; ++l) {
        const int m = OPP.v[l];
        if (m < l) continue;
        const double even = brho + (double)R2_OF(l) * c2E;
        double odd = 0.0;
        if (EX[l] != 0) odd += (double)EX[l] * cjx;
        if (EY[l] != 0) odd += (double)EY[l] * cjy;
        const double ll = lam[l], lm = lam[m];
        lam[l] = (1.0 - om) * ll + (even + odd);
        lam[m] = (1.0 - om) * lm + (even - odd);
    }
    return dtau;
}

// One block sum of a double into partials[blockIdx linear].
template <int T = SITE_THREADS>
__device__ __forceinline__ void block_sum1(double v, double* __restrict__ partials, bool add = false)
{
    double a[1] = {v};
    block_sum_store<1, T>(a, partials + (size_t)blockIdx.y * gridDim.x + blockIdx.x, add);
}

// Threads per block of the reverse step: 256 with FP64 lambda, 64 with FP32
// lambda, where the smaller blocks ran 2.4% (2048x4096), 6% (1024x2048) and
// 8% (512x512) faster over FP32 states; with FP64 lambda they ran 1% slower.
template <typename L>
constexpr int adj_threads() { return sizeof(L) == 4 ? 64 : SITE_THREADS; }

// lambda_{n+1} at site (x, y) (see the header): from a buffer that holds mu
// of the later step (GATHER), or lambda itself at each site (after a seed or
// an explicit set).  Loads are unconditional: in the three rows next to a
// wall the e_y-shifted ones reach into the ghost rows, and those values are
// replaced by 0 below.
template <typename L, bool WALLS, bool GATHER>
__device__ __forceinline__ void load_lambda(const L* __restrict__ buf, const Geo& lg, const WallTable& wt,
                                            int x, int y, double (&lam)[NPOP])
{
    const unsigned yd = (unsigned)y * (unsigned)sizeof(L);
    if (!GATHER) {
        const L* col = buf + lg.origin + (long long)x * lg.cs;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) lam[l] = (double)ld_at(col + (size_t)l * lg.ps, yd);
        return;
    }
    if (!WALLS) {
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            const int xs = wrap_x(x + EX[l], lg.lx);
            int ys = y + EY[l];
            ys = ys < 0 ? ys + lg.ly : (ys >= lg.ly ? ys - lg.ly : ys);
            lam[l] = (double)buf[(size_t)l * lg.ps + lg.origin + (long long)xs * lg.cs + ys];
        }
        return;
    }
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int xs = wrap_x(x + EX[l], lg.lx);
        lam[l] = (double)ld_at(buf + (size_t)l * lg.ps + lg.origin + (long long)xs * lg.cs + EY[l], yd);
    }
    if (y < 3 || y >= lg.ly - 3) {
        const int wall = y < 3 ? 0 : 1;
        const int r = wall == 0 ? y : lg.ly - 1 - y;       // row counted from the wall
        double beta = 0.0;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            if (EY[l] == 0) continue;
            const int en = wall == 0 ? EY[l] : -EY[l];      // hop component into the lattice
            if (-en > r) lam[l] = 0.0;                      // s + e_l lies beyond the wall
            if (en > r) {                                   // a wall slot that mirrors onto s
                const int yw = wall == 0 ? en - 1 - r : lg.ly - en + r;
                const int xw = wrap_x(x + EX[l], lg.lx);
                beta += wt.ew[wall][l] * (double)buf[(size_t)l * lg.ps + lg.origin + (long long)xw * lg.cs + yw];
            }
        }
#pragma unroll
        for (int l = 0; l < NPOP; ++l) lam[l] += beta;
    }
}

// One reverse step at site (x, y): lambda_{n+1} (load_lambda), the gather
// g = bc(propagate(f_n)) of the snapshot f_n, collide^T, and mu stored at the
// site (aligned streaming stores); the block's d/dtau term goes to its slot of
// partials (add: added to the slot, which then sums the terms of many steps).
// (DEV: the device-scope streaming stores, or the plain non-temporal ones
// below DEV_STORES_MIN_BLOCKS_PER_CU blocks per CU)
template <typename S, typename L, bool WALLS, bool GATHER, int T = adj_threads<L>(), bool DEV = true>
__global__ __launch_bounds__(T) void k_adj_collide(
    const S* __restrict__ fn, Geo g, const L* __restrict__ lam_in, L* __restrict__ mu_out, Geo lg,
    AdjArgs a, const double* __restrict__ wall_rho, WallTable wt, double* __restrict__ partials, int add)
{
    const SiteBlock sb = site_block<true, T>(g);
    const int x = sb.x, y = sb.y;
    double dtau = 0.0;
    if (y < g.ly) {
        using Cc = typename Store<S>::C;
        const unsigned yb = (unsigned)y * (unsigned)sizeof(S);
        const unsigned yd = (unsigned)y * (unsigned)sizeof(L);
        double lam[NPOP];
        load_lambda<L, WALLS, GATHER>(lam_in, lg, wt, x, y, lam);
        // the raw gather of f_n (storage precision; unconditional -- wall
        // slots read ghost rows and are replaced below)
        Cc gl[NPOP];
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            int xs = wrap_x(x - EX[l], g.lx);
            if (WALLS) {
                gl[l] = (Cc)ld_at(fn + (size_t)l * g.ps + g.origin + (long long)xs * g.cs - EY[l], yb);
            } else {
                int ys = y - EY[l];
                ys = ys < 0 ? ys + g.ly : (ys >= g.ly ? ys - g.ly : ys);
                gl[l] = (Cc)fn[(size_t)l * g.ps + g.origin + (long long)xs * g.cs + ys];
            }
        }
        // raw moments of g and Lg = sum_l lambda_l g_l, in FP64
        double m0 = 0.0, sx = 0.0, sy = 0.0, s2 = 0.0, Lg = 0.0;
        if (WALLS && (y < 3 || y >= g.ly - 3)) {
#pragma unroll
            for (int l = 0; l < NPOP; ++l) {
                double v = (double)gl[l];
                if (Store<S>::shifted) v += W_SHELL[SHELL[l]];
                if (EY[l] != 0) {
                    const int wall = EY[l] > 0 ? 0 : 1;
                    const int r = wall == 0 ? y : g.ly - 1 - y;
                    const int en = wall == 0 ? EY[l] : -EY[l];
                    if (en > r) v = wt.ew[wall][l] * wall_rho[(wall * 3 + (en - r - 1)) * g.lx + wrap_x(x - EX[l], g.lx)];
                }
                m0 += v;
                if (EX[l] != 0) sx += (double)EX[l] * v;
                if (EY[l] != 0) sy += (double)EY[l] * v;
                if (R2_OF(l) != 0) s2 += (double)R2_OF(l) * v;
                Lg += lam[l] * v;
            }
        } else {
#pragma unroll
            for (int l = 0; l < NPOP; ++l) {
                double v = (double)gl[l];
                if (Store<S>::shifted) v += W_SHELL[SHELL[l]];
                m0 += v;
                if (EX[l] != 0) sx += (double)EX[l] * v;
                if (EY[l] != 0) sy += (double)EY[l] * v;
                if (R2_OF(l) != 0) s2 += (double)R2_OF(l) * v;
                Lg += lam[l] * v;
            }
        }
        dtau = adjoint_site(m0, sx, sy, s2, Lg, lam, a);
        L* mcol = mu_out + lg.origin + (long long)x * lg.cs;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) st_stream<DEV>(mcol + (size_t)l * lg.ps, yd, (L)lam[l]);
    }
    block_sum1<T>(dtau, partials, add != 0);
}

// lambda_l = d(x,y) dT/df_l = d (|xi_l - u|^2 - 2T) / (2 rho), with
// d = dT(x,y) (SEED) or d = T - T_target (LOSS, plus 1/2 d^2 into partials).
template <typename S, typename L, bool LOSS>
__global__ __launch_bounds__(SITE_THREADS) void k_adj_seed_T(const S* __restrict__ fbuf, Geo g, L* __restrict__ lam, Geo lg,
                                                          const double* __restrict__ d_in, double* __restrict__ partials)
{
    const SiteBlock sb = site_block(g);
    const int x = sb.x, y = sb.y;
    double loss = 0.0;
    if (y < g.ly) {
        double rho, ux, uy, T;
        site_macros<S>(fbuf + g.origin + (long long)x * g.cs + y, g.ps, rho, ux, uy, T);
        double d = d_in[(long long)x * g.ly + y];
        if (LOSS) { d = T - d; loss = 0.5 * d * d; }
        const double k = d / (2.0 * rho);
        L* lp = lam + lg.origin + (long long)x * lg.cs + y;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            const double dx = C * EX[l] - ux, dy = C * EY[l] - uy;
            lp[(size_t)l * lg.ps] = (L)(k * (dx * dx + dy * dy - 2.0 * T));
        }
    }
    if (LOSS) block_sum1(loss, partials);
}

// dL/dP from lambda_0 for f_0 = f^eq(rho0(P), 0, T0(P)):
//   T0 = t_mid - t_amp tanh(z), z = (y - y_mid - P) / width, rho0 = p0 / T0,
//   f^eq_l(rho, 0, T) = w_l rho (1 + th K1 + th^2 K3), th = T - 1.
template <typename L, bool WALLS, bool GATHER>
__global__ __launch_bounds__(SITE_THREADS) void k_adj_init_rt(const L* __restrict__ lam_buf, Geo lg, WallTable wt,
                                                           const double* __restrict__ P, RtProfile pr, double* __restrict__ dP)
{
    using K = ShellK<double>;
    const SiteBlock sb = site_block(lg);
    const int x = sb.x, y = sb.y;
    if (y >= lg.ly) return;
    const long long s = (long long)x * lg.ly + y;
    const double th_z = tanh((y - pr.y_mid - P[s]) / pr.width);
    const double T0 = pr.t_mid - pr.t_amp * th_z;
    const double r0 = pr.p0 / T0;
    const double dT = pr.t_amp * (1.0 - th_z * th_z) / pr.width;
    const double dr = -pr.p0 / (T0 * T0) * dT;
    const double th = T0 - 1.0;
    double lam[NPOP];
    load_lambda<L, WALLS, GATHER>(lam_buf, lg, wt, x, y, lam);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int sh = SHELL[l];
        const double Pl = 1.0 + th * (K::k1(sh) + th * K::k3(sh));
        const double dPl = K::k1(sh) + 2.0 * th * K::k3(sh);
        acc += lam[l] * W_SHELL[sh] * (Pl * dr + r0 * dPl * dT);
    }
    dP[s] = acc;
}

// lambda (load_lambda) -> canonical FP64 [37][lx][ly], one thread per site
template <typename L, bool WALLS, bool GATHER>
__global__ __launch_bounds__(SITE_THREADS) void k_lambda_to_canon(const L* __restrict__ buf, Geo lg, WallTable wt,
                                                               double* __restrict__ canon)
{
    const SiteBlock sb = site_block(lg);
    const int x = sb.x, y = sb.y;
    if (y >= lg.ly) return;
    double lam[NPOP];
    load_lambda<L, WALLS, GATHER>(buf, lg, wt, x, y, lam);
#pragma unroll
    for (int l = 0; l < NPOP; ++l) canon[((size_t)l * lg.lx + x) * lg.ly + y] = lam[l];
}

// canonical FP64 [37][lx][ly] -> lambda at each site of a padded buffer of type L
template <typename L>
__global__ __launch_bounds__(256) void k_lambda_from_canon(L* __restrict__ buf, const double* __restrict__ canon, Geo g)
{
    const int nyb = (g.ly + 255) / 256;
    const int l = blockIdx.y, x = (int)(blockIdx.x / (unsigned)nyb);
    const int y = (int)(blockIdx.x % (unsigned)nyb) * 256 + threadIdx.x;
    if (y >= g.ly) return;
    buf[(size_t)l * g.ps + g.origin + (long long)x * g.cs + y] = (L)canon[((size_t)l * g.lx + x) * g.ly + y];
}

}  // namespace lbm
