// The data layouts of the paper's layout study (§4, Table 2), for timing
// propagate and collide on each: FP64 populations of an lx x ly lattice,
// periodic in x and y, with no halo or padding.
//
// Population l of site (x, y):
//   AOS     ((x ly + y) 37 + l)                    all 37 of a site together
//   SOA     ((l lx + x) ly + y)                    one array per population
//   CSOA    (((l lx + x) M + i) VL + k)            y = k M + i, M = ly / VL
//   CAOSOA  (((x M + i) 37 + l) VL + k)            y = k M + i
// The clustered layouts split every column into VL partitions of M rows; a
// cluster packs the rows at offset i of all VL partitions, so a shift of y by
// e_y moves whole clusters (i -> i - e_y) except where i - e_y leaves
// [0, M), where it also moves one lane (k -> k -+ 1).  CSOA keeps one array per
// population; CAOSOA keeps the 37 clusters of a cluster-site together.  With
// VL = 1, CSOA is SOA and CAOSOA is AOS.
//
// The kernels are deliberately generic (one 8-byte element per thread in
// propagate, one site per thread in collide), so that the layouts, not kernel
// tuning, decide the differences.  The library's own step kernels use the
// padded layouts of lbm_kernels.hpp instead.
#pragma once
#include "lbm_kernels.hpp"

namespace lbm {

enum StudyLayout : int { ST_AOS = 0, ST_SOA = 1, ST_CSOA = 2, ST_CAOSOA = 3 };

struct StudyGeo {
    int lx, ly;
    int vl, lvl;   // cluster width (1 for AOS and SOA) and its log2
    int m;         // rows per partition, ly / vl
};

// element index of population l at column x, lane k, partition row i
template <int LAY>
__host__ __device__ __forceinline__ size_t st_index(const StudyGeo& g, int l, int x, int k, int i)
{
    if constexpr (LAY == ST_AOS) return ((size_t)x * g.ly + i) * NPOP + l;
    else if constexpr (LAY == ST_SOA) return ((size_t)l * g.lx + x) * g.ly + i;
    else if constexpr (LAY == ST_CSOA) return (((size_t)l * g.lx + x) * g.m + i) * g.vl + k;
    else return (((size_t)x * g.m + i) * NPOP + l) * g.vl + k;
}

// Contiguous runs of memory that propagate walks in order: one (population,
// column) array for SOA and CSOA, one column of all populations for AOS and
// CAOSOA.
template <int LAY>
__host__ __device__ __forceinline__ constexpr bool st_per_population()
{
    return LAY == ST_SOA || LAY == ST_CSOA;
}

constexpr int ST_THREADS = 256;

// propagate (eq. (4), pull): dst_l(x, y) = src_l(x - e_x, y - e_y), both
// periodic.  One destination element per thread, in destination memory
// order; grid = segments x chunks of ST_THREADS elements.
template <int LAY>
__global__ __launch_bounds__(ST_THREADS) void k_study_propagate(const double* __restrict__ src,
                                                                double* __restrict__ dst, StudyGeo g,
                                                                unsigned nch)
{
    const unsigned seg = blockIdx.x / nch, ch = blockIdx.x % nch;
    const unsigned seglen = st_per_population<LAY>() ? (unsigned)g.ly : (unsigned)g.ly * NPOP;
    const unsigned j = ch * ST_THREADS + threadIdx.x;
    if (j >= seglen) return;
    int l, x, k, i;
    if constexpr (st_per_population<LAY>()) {
        l = (int)(seg / (unsigned)g.lx);
        x = (int)(seg % (unsigned)g.lx);
        k = (int)(j & (unsigned)(g.vl - 1));
        i = (int)(j >> g.lvl);
    } else {
        x = (int)seg;
        k = (int)(j & (unsigned)(g.vl - 1));
        const unsigned r = j >> g.lvl;
        i = (int)(r / NPOP);
        l = (int)(r - (unsigned)i * NPOP);
    }
    const int ex = c_hops.ex[l], ey = c_hops.ey[l];
    const int xs = wrap_x(x - ex, g.lx);
    int is = i - ey, ks = k;
    if (is < 0) { is += g.m; ks = ks == 0 ? g.vl - 1 : ks - 1; }
    else if (is >= g.m) { is -= g.m; ks = ks == g.vl - 1 ? 0 : ks + 1; }
    const double v = __builtin_nontemporal_load(src + st_index<LAY>(g, l, xs, ks, is));
    // the destination is element j of segment seg (memory order), stored
    // with the library's streaming store from the segment's start
    st_nt(dst + (size_t)seg * seglen, j * 8u, v);
}

// collide in place, one site per thread.  Threads of a block take the sites
// of one column in (partition row, lane) order with the lane fastest, so a
// wave's loads of one population are VL-element runs (contiguous for SOA and
// CSOA, 37 VL elements apart for CAOSOA, 37 elements apart for AOS).
template <int LAY>
__global__ __launch_bounds__(SITE_THREADS) void k_study_collide(double* __restrict__ buf, StudyGeo g,
                                                                CollideArgs args, unsigned nch)
{
    const unsigned x = blockIdx.x / nch, ch = blockIdx.x % nch;
    const unsigned s = ch * SITE_THREADS + threadIdx.x;   // site of column x, in (i, k) order
    if (s >= (unsigned)g.ly) return;
    const int k = (int)(s & (unsigned)(g.vl - 1)), i = (int)(s >> g.lvl);
    double* col = buf + st_index<LAY>(g, 0, (int)x, 0, 0);
    // the site's offset from its column's start, the same for every population
    const size_t so = st_index<LAY>(g, 0, (int)x, k, i) - st_index<LAY>(g, 0, (int)x, 0, 0);
    const size_t stride = st_index<LAY>(g, 1, 0, 0, 0);    // distance between populations
    double f[NPOP];
#pragma unroll
    for (int l = 0; l < NPOP; ++l) f[l] = __builtin_nontemporal_load(col + so + l * stride);
    collide_site<double, false>(f, args);
    // A wave's stores of one population are one 512-byte run in SOA and CSOA,
    // which take the library's streaming store.  In AOS they are 8-byte
    // pieces 296 B apart, which that store writes through the L2 one at a
    // time (AOS collide: 9.5 -> 31.5 ms at 2160x8192); AOS and CAOSOA (runs
    // of VL elements 37 VL apart: -3% to +3% with it) keep plain
    // non-temporal stores, which the L2 merges into whole lines.
    if constexpr (st_per_population<LAY>()) {
#pragma unroll
        for (int l = 0; l < NPOP; ++l) st_nt(col + l * stride, (unsigned)(so * 8), f[l]);
    } else {
#pragma unroll
        for (int l = 0; l < NPOP; ++l) __builtin_nontemporal_store(f[l], col + so + l * stride);
    }
}

// canonical FP64 [37][lx][ly] <-> layout, one element per thread
template <int LAY, bool TO_LAYOUT>
__global__ __launch_bounds__(256) void k_study_convert(double* __restrict__ buf, double* __restrict__ canon,
                                                       StudyGeo g, size_t n)
{
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (size_t)gridDim.x * 256) {
        const int y = (int)(c % (size_t)g.ly);
        const size_t t = c / (size_t)g.ly;
        const int x = (int)(t % (size_t)g.lx), l = (int)(t / (size_t)g.lx);
        const size_t b = st_index<LAY>(g, l, x, y / g.m, y % g.m);
        if (TO_LAYOUT) buf[b] = canon[c];
        else canon[c] = buf[b];
    }
}

}  // namespace lbm
