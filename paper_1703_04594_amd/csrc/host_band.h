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
    int gr;   // ghost rows above and below each segment
};

// One halo message between the two parts of a split lattice: whole padded
// population segments (ps values each, in list order), then the six wall
// rows (y = 0, 1, 2, ly-3, ly-2, ly-1) of further populations.  A halo
// column needs only the populations whose hop reaches the receiver's own
// columns from it, plus, for the wall rule's mirror densities, the wall rows
// of the others.  Columns are those of the lattice that packs or unpacks.
struct SeamList {
    int nseg, nwall;
    int seg_col[64];
    unsigned char seg_pop[64];
    int wall_col[256];
    unsigned char wall_pop[256];
};

inline size_t seam_values(const SeamList& s, long long ps) { return (size_t)s.nseg * ps + (size_t)s.nwall * 6; }

// pack: the listed data of buf -> stage; else stage -> buf.
void seam_copy(double* buf, const BandGeo& g, const SeamList& s, double* stage, bool pack, int nthreads);

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
