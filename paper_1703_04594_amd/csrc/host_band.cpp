// host_band.cpp -- one fused D2Q37 step over a band of columns, on host cores.
//
// The arithmetic is the GPU step's (section 3: moments of eq. (2), the
// gravity shift, the 4th-order Hermite equilibrium in Horner form in
// a = xi_l . u, BGK relaxation of eq. (1); the library's wall rule), laid out
// for SIMD: every thread takes whole columns, and every per-site quantity is
// a vector over a block of B consecutive rows (the rows of one population
// segment are contiguous, so a block's loads and stores are vector moves).
#include "host_band.h"

#include <immintrin.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <utility>

#include "d2q37_tables.h"

namespace lbm_host {
namespace {

using namespace d2q37;

constexpr int B = 8;   // rows per block
constexpr int PF = 32;  // prefetch distance, rows
// B doubles: two AVX2 registers (one AVX-512 register where available)
typedef double vb __attribute__((vector_size(B * sizeof(double))));

// Compile-time loop: f(std::integral_constant<int, i>) for i = 0 .. N-1, so
// that hop-table lookups inside are constants.
template <class F, int... I>
inline void static_for_(F& f, std::integer_sequence<int, I...>) { (f(std::integral_constant<int, I>{}), ...); }
template <int N, class F>
inline void static_for(F&& f) { static_for_(f, std::make_integer_sequence<int, N>{}); }

// |xi_l|^2 as the moments define it: xi_l = c e_l rounded per component, then
// squared and summed (the GPU step's FP64 constants; constant-evaluated, so
// every operation rounds once).
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

// Shell constants of the Hermite coefficients (x2 = |xi|^2 of the shell):
//   A0 - 1 = u2 (-1/2 + u2/8) + th (k1 + u2 k2 + th k3),  A1 = 1 - u2/2 + th k4,
//   A2 = 1/2 - u2/4 + th k5.
struct ShellC { double k1, k2, k3, k4, k5; };
constexpr ShellC shell_c(int s)
{
    const double x2 = xi2_of_shell(s);
    return ShellC{(x2 - 2.0) / 2.0, (4.0 - x2) / 4.0, (x2 * x2 - 8.0 * x2 + 8.0) / 8.0, (x2 - 4.0) / 2.0,
                  (x2 - 6.0) / 4.0};
}

inline int wrap(int x, int lx) { return x < 0 ? x + lx : (x >= lx ? x - lx : x); }

// BGK collision of B sites in place.
inline void collide_block(vb (&f)[NPOP], const BandArgs& a)
{
    vb m0 = {}, sx = {}, sy = {}, e2 = {};
    static_for<NPOP>([&](auto lc) {
        constexpr int l = decltype(lc)::value;
        m0 += f[l];
        if constexpr (EX[l] != 0) sx += double(EX[l]) * f[l];
        if constexpr (EY[l] != 0) sy += double(EY[l]) * f[l];
        if constexpr (l != 0) {
            constexpr double x2 = xi2_of_pop(l);
            e2 += x2 * f[l];
        }
    });
    const vb rho = m0;
    const vb inv = 1.0 / rho;
    const vb ux = C * sx * inv;
    const vb uy0 = C * sy * inv;
    const vb th = (e2 * inv - (ux * ux + uy0 * uy0)) * 0.5 - 1.0 + a.grav_th;
    const vb uy = uy0 + a.tau_g;
    const vb u2 = ux * ux + uy * uy;
    const vb cux = C * ux, cuy = C * uy;
    const vb b1 = 1.0 - 0.5 * u2;
    const vb b2 = 0.5 - 0.25 * u2;
    const vb b0m1 = u2 * (-0.5 + 0.125 * u2);
    const double om = a.omega;
    static_for<NSHELL>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr ShellC k = shell_c(s);
        const vb A0m1 = b0m1 + th * (k.k1 + u2 * k.k2 + th * k.k3);
        const vb A1 = b1 + th * k.k4;
        const vb A2 = b2 + th * k.k5;
        const vb wrho = W_SHELL[s] * rho;
        static_for<NPOP>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            if constexpr (SHELL[l] == s) {
                vb pm;
                if constexpr (l == 0) {
                    pm = A0m1;
                } else {
                    vb av;
                    if constexpr (EX[l] != 0 && EY[l] != 0) av = double(EX[l]) * cux + double(EY[l]) * cuy;
                    else if constexpr (EX[l] != 0) av = double(EX[l]) * cux;
                    else av = double(EY[l]) * cuy;
                    vb t = av * (1.0 / 24.0) + 1.0 / 6.0;
                    t = t * av + A2;
                    t = t * av + A1;
                    pm = t * av + A0m1;
                }
                f[l] = f[l] + om * (wrho * (1.0 + pm) - f[l]);
            }
        });
    });
}

}  // namespace

void fused_step(const double* src_c, double* dst, const BandGeo& g, const BandArgs& a, double* wall_rho, int nthreads)
{
    double* src = const_cast<double*>(src_c);   // y ghost rows are refreshed in place (periodic y)
    const int lx = g.lx, ly = g.ly;
    // row 0 of every segment is 128-byte aligned relative to the buffer, so
    // blocks of B rows are whole aligned lines when the buffer is
    const bool nt = ((uintptr_t)dst % 64) == 0;
#pragma omp parallel num_threads(nthreads)
    {
        // 1. per column: wall-row densities (walls) or y ghost rows (periodic)
#pragma omp for schedule(static)
        for (int x = 0; x < lx; ++x) {
            double* col = src + g.origin + (long long)x * g.cs;
            if (a.walls) {
                for (int wall = 0; wall < 2; ++wall)
                    for (int k = 0; k < 3; ++k) {
                        const int y = wall == 0 ? k : ly - 1 - k;
                        double r = 0.0;
                        for (int l = 0; l < NPOP; ++l) r += col[l * g.ps + y];
                        wall_rho[(wall * 3 + k) * lx + x] = r;
                    }
            } else {
                for (int l = 0; l < NPOP; ++l) {
                    double* p = col + l * g.ps;
                    for (int k = 1; k <= 3; ++k) {
                        p[-k] = p[ly - k];
                        p[ly - 1 + k] = p[k - 1];
                    }
                }
            }
        }
        // 2. pull gather, wall rule, collide; one column per iteration
#pragma omp for schedule(static)
        for (int x = 0; x < lx; ++x) {
            const double* sp[NPOP];
            for (int l = 0; l < NPOP; ++l)
                sp[l] = src + l * g.ps + g.origin + (long long)wrap(x - EX[l], lx) * g.cs - EY[l];
            double* dcol = dst + g.origin + (long long)x * g.cs;
            for (int y0 = 0; y0 < ly; y0 += B) {
                vb f[NPOP];
                // the last block reads past row ly - 1 into the ghost rows;
                // those lanes are computed and discarded
                for (int l = 0; l < NPOP; ++l) std::memcpy(&f[l], sp[l] + y0, sizeof(vb));
                // 74 concurrent streams (37 read, 37 written) are more than
                // the hardware prefetchers follow: fetch PF rows ahead
                for (int l = 0; l < NPOP; ++l) {
                    __builtin_prefetch(sp[l] + y0 + PF, 0, 3);
                    if (!nt) __builtin_prefetch(dcol + l * g.ps + y0 + PF, 1, 3);
                }
                if (a.walls && (y0 < 3 || y0 + B > ly - 3)) {
                    for (int b = 0; b < B; ++b) {
                        const int y = y0 + b;
                        if (y >= ly || (y >= 3 && y < ly - 3)) continue;
                        const int wall = y < 3 ? 0 : 1;
                        const int r = wall == 0 ? y : ly - 1 - y;   // row counted from the wall
                        for (int l = 0; l < NPOP; ++l) {
                            const int en = wall == 0 ? EY[l] : -EY[l];   // hop component into the lattice
                            if (en > r)   // the pull source lies beyond the wall: its mirror's density
                                f[l][b] = a.ew[wall][l] * wall_rho[(wall * 3 + (en - r - 1)) * lx + wrap(x - EX[l], lx)];
                        }
                    }
                }
                collide_block(f, a);
                const int nb = std::min(B, ly - y0);
                if (nb == B && nt) {
                    // whole 64-byte lines, written once: streaming stores
                    for (int l = 0; l < NPOP; ++l) {
                        double* q = dcol + l * g.ps + y0;
                        _mm256_stream_pd(q, __m256d{f[l][0], f[l][1], f[l][2], f[l][3]});
                        _mm256_stream_pd(q + 4, __m256d{f[l][4], f[l][5], f[l][6], f[l][7]});
                    }
                } else if (nb == B) {
                    for (int l = 0; l < NPOP; ++l) std::memcpy(dcol + l * g.ps + y0, &f[l], sizeof(vb));
                } else {
                    for (int l = 0; l < NPOP; ++l)
                        for (int b = 0; b < nb; ++b) dcol[l * g.ps + y0 + b] = f[l][b];
                }
            }
        }
        _mm_sfence();   // streaming stores visible before the region ends
    }
}

void seam_copy(double* buf, const BandGeo& g, const SeamList& s, double* stage, bool pack, int nthreads)
{
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int j = 0; j < s.nseg; ++j) {
        double* seg = buf + g.origin - g.gr + (long long)s.seg_col[j] * g.cs + (long long)s.seg_pop[j] * g.ps;
        double* st = stage + (size_t)j * g.ps;
        if (pack) std::memcpy(st, seg, sizeof(double) * g.ps);
        else std::memcpy(seg, st, sizeof(double) * g.ps);
    }
    double* st = stage + (size_t)s.nseg * g.ps;
    for (int e = 0; e < s.nwall * 6; ++e) {
        const int w = e / 6, r = e % 6;
        const int y = r < 3 ? r : g.ly - 6 + r;
        double* q = buf + g.origin + (long long)s.wall_col[w] * g.cs + (long long)s.wall_pop[w] * g.ps + y;
        if (pack) st[e] = *q;
        else *q = st[e];
    }
}

}  // namespace lbm_host
