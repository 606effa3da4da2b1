// host_band.h -- the host's part of a lattice shared between host cores and
// the GPU (section 5: border columns on the host, the bulk on the
// accelerator, halos of three columns exchanged every step).  Plain C++,
// built with the host compiler; no HIP.
#pragma once
#include <cstddef>

namespace lbm_host {

// A band of lx columns stored like the GPU library's FP64 column layout:
// population l of site (x, y) at l*ps + origin + x*cs + y, with ghost rows
// above and below every segment.  The band is periodic over its own lx
// columns; the caller overwrites its outer columns (the halos) with the
// neighbour's values after every step.
struct BandGeo {
    int lx, ly;
    long long ps, cs, origin;
};

struct BandArgs {
    double omega, tau_g, grav_th;   // 1/tau, tau g_y, tau (1 - tau) g_y^2 / 2
    bool walls;
    double ew[2][37];               // f^eq_l(1, 0, T_wall) of the bottom and top walls
};

// One fused step src -> dst (pull streaming of eq. (4), the wall rule,
// collide), on nthreads host threads.  wall_rho: scratch of 6 * lx doubles.
void fused_step(const double* src, double* dst, const BandGeo& g, const BandArgs& a, double* wall_rho,
                int nthreads);

}  // namespace lbm_host
