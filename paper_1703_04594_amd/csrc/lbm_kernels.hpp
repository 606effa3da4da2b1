// lbm_kernels.hpp -- gfx950 kernels of the D2Q37 step (forward).
//
// Storage: two population buffers of padded columns.  A column segment holds
// one population of one lattice column, y fastest (the paper's column-major
// choice, section 4), padded with G ghost rows on both sides (G * sizeof(S) =
// 128 B, so interior row 0 of every segment is 128-byte aligned); there are 3
// halo columns on both sides (hops reach 3 sites).  Population l of site
// (x, y) sits at  l * ps + origin + x * cs + y  with either
//   planes:  ps = one whole plane, cs = lyp       (structure of arrays), or
//   columns: ps = lyp,             cs = 37 * lyp  (the 37 segments of a column
//            contiguous, so the 37 streams of a site lie within one column).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_site.hpp"

namespace lbm {

struct Geo {
    int lx, ly;       // interior sites
    int lyp;          // padded column-segment length (elements)
    int g;            // ghost rows below / above (elements)
    long long ps;     // stride between populations (elements)
    long long cs;     // stride between columns (elements)
    long long origin; // element index of population 0 at site (0, 0)
    long long total;  // elements per buffer
};

constexpr int HALO_X = 3;

// Geometry of a padded population buffer of lx x ly sites with elem-byte
// values: planes (structure of arrays) or columns layout.
inline Geo padded_geo(int lx, int ly, size_t elem, bool planes)
{
    auto up = [](size_t v, size_t a) { return (v + a - 1) / a * a; };
    Geo g;
    g.lx = lx;
    g.ly = ly;
    g.g = (int)(128 / elem);                             // 128-byte aligned row 0
    const int col_align = (int)(128 / elem);
    g.lyp = (int)up((size_t)ly + 2 * g.g, (size_t)col_align);
    // An odd number of 128-byte lines per column segment.  With an even
    // count, segment strides near a power of two (ly = 8192 in FP64: 514
    // lines, 64 KiB + 256 B) slowed propagate from 6.3 to 5.3 TB/s; one more
    // line restores it, and costs nothing measurable on other shapes.
    if ((size_t)g.lyp * elem / 128 % 2 == 0) g.lyp += col_align;
    const long long ncol = lx + 2 * HALO_X;
    if (planes) {
        g.cs = g.lyp;
        g.ps = (long long)up((size_t)ncol * g.lyp * elem, 256) / (long long)elem;
        g.total = NPOP * g.ps;
    } else {
        g.ps = g.lyp;
        g.cs = (long long)NPOP * g.lyp;
        g.total = ncol * g.cs;
    }
    g.origin = (long long)HALO_X * g.cs + g.g;
    return g;
}

struct HopTable { int ex[NPOP]; int ey[NPOP]; };
constexpr HopTable make_hops()
{
    HopTable t{};
    for (int l = 0; l < NPOP; ++l) { t.ex[l] = EX[l]; t.ey[l] = EY[l]; }
    return t;
}
__constant__ HopTable c_hops = make_hops();

// Wall slots: after propagate, slot (l, row r of a wall) pulls from outside
// the lattice iff the hop towards the interior, e_n = ey (bottom) or -ey
// (top), exceeds r.  The mirror fluid row is k = e_n - r - 1.  15 + 8 + 3
// slots per wall and column.
constexpr int NSLOT = 52;
struct SlotTable { int l[NSLOT]; int row[NSLOT]; int k[NSLOT]; int wall[NSLOT]; };
constexpr SlotTable make_slots()
{
    SlotTable t{};
    int n = 0;
    for (int wall = 0; wall < 2; ++wall)
        for (int r = 0; r < 3; ++r)
            for (int l = 0; l < NPOP; ++l) {
                const int en = wall == 0 ? EY[l] : -EY[l];
                if (en > r) { t.l[n] = l; t.row[n] = r; t.k[n] = en - r - 1; t.wall[n] = wall; ++n; }
            }
    return t;
}
static_assert(make_slots().l[NSLOT - 1] != 0, "52 wall slots");
__constant__ SlotTable c_slots = make_slots();

// f^eq_l(1, 0, T_wall) of both walls, and the weights (for shifted storage).
struct WallTable { double ew[2][NPOP]; double w[NPOP]; };

template <typename S> struct Store;
template <> struct Store<double> { using C = double; static constexpr bool shifted = false; };
template <> struct Store<float>  { using C = float;  static constexpr bool shifted = true; };

__device__ __forceinline__ int wrap_x(int xs, int lx)
{
    return xs < 0 ? xs + lx : (xs >= lx ? xs - lx : xs);
}

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin by
// linear id.  Site kernels use a 1-D grid and renumber hardware block b as
// L = k q + min(k, r) + i  (k = b mod 8, i = b div 8, N = 8 q + r blocks), a
// bijection that hands each XCD one contiguous run of lattice chunks, so the
// cache lines shared by neighbouring chunks (shifted gathers and pushes) are
// reused in the same L2.
constexpr int NXCD = 8;
constexpr int SITE_THREADS = 256;
__device__ __forceinline__ int xcd_block(int b, int n)
{
    const int k = b % NXCD, i = b / NXCD;
    const int q = n / NXCD, r = n % NXCD;
    return k * q + (k < r ? k : r) + i;
}

// Site kernels: block L covers sites y in [bx * T, ...) of column x, T the
// block's threads (SITE_THREADS, except the reverse step with FP32 lambda).
// (Measured: the renumbering gains 5% on the FP64 step and 14% on the
// adjoint step, but costs ~1% on the FP32 step, which therefore keeps the
// hardware order.)
struct SiteBlock { int x, y; };
template <bool REMAP = true, int T = SITE_THREADS>
__device__ __forceinline__ SiteBlock site_block(const Geo& g)
{
    const int nyb = (g.ly + T - 1) / T;
    const int L = REMAP ? xcd_block(blockIdx.x, nyb * g.lx) : (int)blockIdx.x;
    return SiteBlock{L / nyb, (L % nyb) * T + (int)threadIdx.x};
}

// Plane access as (block-uniform base pointer) + (per-thread 32-bit byte
// offset): the base lives in scalar registers and one vector offset serves all
// 37 planes, so no 64-bit per-plane vector addresses are kept alive.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, unsigned byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
// Non-temporal form of ld_at, for data read exactly once with no reuse by
// neighbouring workgroups (in-place collide): 8-9% faster there.  Gathers
// keep temporal loads: lines straddled by their e_y shift are shared with the
// neighbouring wave.
template <typename T>
__device__ __forceinline__ T ld_nt(const T* base, unsigned byte_off)
{
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off));
}
// Streaming store of a 4-, 8- or 16-byte value at base + byte_off, base
// block-uniform (it becomes a buffer resource in scalar registers).  The
// store carries the non-temporal hint and device scope (cache policy nt sc1),
// so it is written through the XCD's L2 without being kept there.  Against
// plain non-temporal stores (same launches, bitwise-equal results, 2048x4096,
// two runs each, ms) it took propagate from 0.772-0.778 to 0.766-0.767 (FP64)
// and 0.389-0.390 to 0.382-0.383 (FP32), the in-place FP32 collide from 0.418
// to 0.396, the reverse step with FP64 lambda from 1.082-1.083 to 1.066-1.068,
// and the fused steps 0.3-0.5% lower; the fused FP64 step's access pattern
// alone ran 0.831 -> 0.811.  Stores without nt, or with sc1 alone, were 5-8%
// slower than nt.  Below 2048x4096 device scope costs the fused and reverse
// steps time instead, so those take the store form as a template parameter
// (st_stream), chosen per lattice at launch; a uniform flag tested before
// each store instead kept all 37 values live across the branches (FP32
// step: 62 -> 126 VGPRs).
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
// cache-policy bits of a gfx950 buffer instruction: nt (non-temporal) and
// sc1 (scope bit 1: device scope)
constexpr int CPOL_NT = 2, CPOL_SC1 = 16;
constexpr int STORE_CPOL_NT_SC1 = CPOL_NT | CPOL_SC1;
// Raw buffer descriptor (stride 0): num_records is a byte count, here the
// whole 32-bit offset range; word 3 sets the 32-bit data format (field value 4
// at bit 15), as raw accesses take their size from the instruction.
constexpr int RAW_BUFFER_ALL_BYTES = -1;
constexpr int RAW_BUFFER_WORD3 = 0x00020000;
template <typename T>
__device__ __forceinline__ void st_nt(T* base, unsigned byte_off, T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "4, 8 or 16-byte stores");
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(base, 0, RAW_BUFFER_ALL_BYTES, RAW_BUFFER_WORD3);
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0,
                                              STORE_CPOL_NT_SC1);
    else if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)byte_off, 0,
                                              STORE_CPOL_NT_SC1);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, (int)byte_off, 0,
                                               STORE_CPOL_NT_SC1);
}
// The fused step's and reverse step's stores: the device-scope streaming
// store above (DEV), or the plain non-temporal store, which their
// instantiations for lattices below DEV_STORES_MIN_BLOCKS_PER_CU blocks per CU
// use.
template <bool DEV, typename T>
__device__ __forceinline__ void st_stream(T* base, unsigned byte_off, T v)
{
    if constexpr (DEV) st_nt(base, byte_off, v);
    else __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off));
}
// Device scope pays on large lattices only (see st_nt): the fused and reverse
// steps take it from this many site blocks (of SITE_THREADS) per CU on,
// i.e. from 8,388,608 sites (2048x4096) on a 256-CU GPU.  A/B of the two
// store forms on one box (fused FP64 step / reverse step with FP64 lambda,
// us per step, two runs each): 256x128 8.4 / 12.6 with plain non-temporal
// stores against 9.2 / 13.5 at device scope, 512x512 28.2 / 44.0 against
// 28.8-29.3 / 44.9, 1024x1024 119 / 183 against 123 / 186, 2048x2048 440 /
// 559 against 446 / 557, 2048x4096 835-837 / 1082 against 833-834 / 1067.
constexpr unsigned DEV_STORES_MIN_BLOCKS_PER_CU = 128;
inline bool dev_stores_for(size_t nb256, int ncu)
{
    return ncu > 0 && nb256 >= (size_t)DEV_STORES_MIN_BLOCKS_PER_CU * (size_t)ncu;
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, unsigned byte_off, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// ---------------------------------------------------------------------------
// propagate: dst_l(x, y) = src_l(x - ex_l, y - ey_l).  One block streams a
// chunk of one column of one plane; each thread moves UNROLL vectors of VEC
// elements.  Stores are aligned; loads are shifted by ey elements (unaligned
// vector loads are legal on CDNA for dword-aligned addresses).
// ---------------------------------------------------------------------------
template <typename S, int VEC> struct VecT;
template <> struct VecT<double, 1> { typedef double T __attribute__((ext_vector_type(1), aligned(8))); };
template <> struct VecT<double, 2> { typedef double T __attribute__((ext_vector_type(2), aligned(8))); };
template <> struct VecT<float, 2> { typedef float T __attribute__((ext_vector_type(2), aligned(4))); };
template <> struct VecT<float, 4> { typedef float T __attribute__((ext_vector_type(4), aligned(4))); };
template <typename S, int VEC> struct VecA;
template <> struct VecA<double, 1> { typedef double T __attribute__((ext_vector_type(1))); };
template <> struct VecA<double, 2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct VecA<float, 2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct VecA<float, 4> { typedef float T __attribute__((ext_vector_type(4))); };

// propagate: 256 threads, one 16-byte vector each, so a workgroup moves 4 KB
// of one segment.  Loads and stores are both non-temporal (each byte is read
// once and written once).  Workgroups are numbered linearly, chunk fastest,
// then the population index (COLS layout: the 37 segments of a column are
// contiguous) or the column (planes layout), so consecutive workgroups stream
// consecutive memory, and they run in hardware order (all XCDs sweep the same
// region of memory together).  Measured on the 2048x4096 lattice, this beat
// 1, 2, 8 and 16 KB workgroups, temporal loads, an XCD-contiguous
// renumbering and a 3-D (chunk, population, column) grid.
constexpr int PROP_THREADS = 256;
constexpr int PROP_UNROLL = 1;
// widest x dimension of the propagate grid in workgroups: a dispatch holds
// each dimension's work-item count in 32 bits.  Larger launches add rows,
// still dispatched in linear order; rows of 2^20 workgroups measured 9%
// slower than one row at 2048x8192.
constexpr unsigned PROP_GRID_X = 0xffffffffu / PROP_THREADS;

template <typename S, int VEC, int UNROLL, bool WRAP, bool COLS>
__global__ __launch_bounds__(PROP_THREADS) void k_propagate(const S* __restrict__ src, S* __restrict__ dst, Geo g,
                                                            unsigned nblk)
{
    using VU = typename VecT<S, VEC>::T;
    using VA = typename VecA<S, VEC>::T;
    const unsigned L = blockIdx.y * gridDim.x + blockIdx.x;
    if (L >= nblk) return;
    const int nch = (g.ly + PROP_THREADS * VEC * UNROLL - 1) / (PROP_THREADS * VEC * UNROLL);
    const int ch = (int)(L % (unsigned)nch);
    const unsigned rest = L / (unsigned)nch;
    const int l = (int)(COLS ? rest % NPOP : rest / (unsigned)g.lx);
    const int x = (int)(COLS ? rest / NPOP : rest % (unsigned)g.lx);
    const int ex = c_hops.ex[l], ey = c_hops.ey[l];
    int xs = x - ex;
    if (WRAP) xs = wrap_x(xs, g.lx);
    const S* sp = src + (size_t)l * g.ps + g.origin + (long long)xs * g.cs - ey;
    S* dp = dst + (size_t)l * g.ps + g.origin + (long long)x * g.cs;
    const int y0 = ch * (PROP_THREADS * VEC * UNROLL) + threadIdx.x * VEC;
    VU v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int y = y0 + u * PROP_THREADS * VEC;
        if (y < g.ly) v[u] = __builtin_nontemporal_load(reinterpret_cast<const VU*>(sp + y));
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int y = y0 + u * PROP_THREADS * VEC;
        if (y < g.ly) st_nt<VA>(reinterpret_cast<VA*>(dp), (unsigned)y * (unsigned)sizeof(S), (VA)v[u]);
    }
}

// x halos for LBM_X_HALO: copy whole padded columns into the 3 halo columns
// of each side (only the planes whose hop needs them).  Thread per element.
template <typename S>
__global__ __launch_bounds__(256) void k_fill_x_halo(S* __restrict__ buf, Geo g)
{
    const int l = blockIdx.z;
    const int ex = c_hops.ex[l];
    const int d = blockIdx.y;          // 0..2 -> halo column depth d + 1
    if (ex == 0 || d >= (ex > 0 ? ex : -ex)) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.lyp) return;
    S* p = buf + (size_t)l * g.ps + g.origin - g.g + i;
    const int to = ex > 0 ? -(d + 1) : g.lx + d;
    const int from = ex > 0 ? g.lx - (d + 1) : d;
    p[(long long)to * g.cs] = p[(long long)from * g.cs];
}

// y ghost rows for LBM_Y_PERIODIC: rows [-3, 0) <- [ly-3, ly), [ly, ly+3) <- [0, 3).
template <typename S>
__global__ __launch_bounds__(256) void k_fill_y_ghosts(S* __restrict__ buf, Geo g)
{
    const int l = blockIdx.y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g.lx * 6) return;
    const int x = t / 6, r = t % 6;
    S* p = buf + (size_t)l * g.ps + g.origin + (long long)x * g.cs;
    if (r < 3) p[r - 3] = p[g.ly - 3 + r];
    else p[g.ly + r - 3] = p[r - 3];
}

// Density of the 3 rows next to each wall (FP64), for the wall rule.
// wall_rho[(wall * 3 + k) * lx + x]: bottom row k, top row ly-1-k.
template <typename S>
__global__ __launch_bounds__(256) void k_wall_density(const S* __restrict__ buf, Geo g, double* __restrict__ wall_rho)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= 6 * g.lx) return;
    const int x = t % g.lx, wk = t / g.lx;
    const int wall = wk / 3, k = wk % 3;
    const int y = wall == 0 ? k : g.ly - 1 - k;
    const S* p = buf + g.origin + (long long)x * g.cs + y;
    double r = 0.0;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) r += (double)p[(size_t)l * g.ps];
    wall_rho[t] = Store<S>::shifted ? 1.0 + r : r;
}

// Wall rule on the current buffer (split step): thread per (column, slot).
template <typename S>
__global__ __launch_bounds__(256) void k_bc_apply(S* __restrict__ dst, Geo g, const double* __restrict__ wall_rho, WallTable wt)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= NSLOT * g.lx) return;
    const int j = t % NSLOT, x = t / NSLOT;
    const int l = c_slots.l[j], wall = c_slots.wall[j];
    const int y = wall == 0 ? c_slots.row[j] : g.ly - 1 - c_slots.row[j];
    const int xs = wrap_x(x - c_hops.ex[l], g.lx);
    double v = wt.ew[wall][l] * wall_rho[(wall * 3 + c_slots.k[j]) * g.lx + xs];
    if (Store<S>::shifted) v -= wt.w[l];
    dst[(size_t)l * g.ps + g.origin + (long long)x * g.cs + y] = (S)v;
}

// ---------------------------------------------------------------------------
// collide: one thread per site, in place.
// ---------------------------------------------------------------------------

// Density of a site from its just-written populations, summed in population
// order in FP64 exactly as k_wall_density sums them, into the wall-density
// table of the next step (rows 0..2 and ly-3..ly-1 only).
template <typename S, typename Cc>
__device__ __forceinline__ void store_wall_density(const Cc (&f)[NPOP], const Geo& g, int x, int y,
                                                   double* __restrict__ wall_rho_out)
{
    if (y < 3 || y >= g.ly - 3) {
        double r = 0.0;
#pragma unroll
        for (int l = 0; l < NPOP; ++l) r += (double)(S)f[l];
        const int wk = y < 3 ? y : 3 + (g.ly - 1 - y);
        wall_rho_out[wk * g.lx + x] = Store<S>::shifted ? 1.0 + r : r;
    }
}

// WIDE = false: FP32 storage collided with FP32 moment sums (collide_site).
template <typename S, bool WALLS, bool WIDE = true>
__global__ __launch_bounds__(SITE_THREADS) void k_collide(S* __restrict__ buf, Geo g, CollideArgs args,
                                                       double* __restrict__ wall_rho_out)
{
    using Cc = typename Store<S>::C;
    const SiteBlock sb = site_block<sizeof(S) == 8>(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    S* col = buf + g.origin + (long long)x * g.cs;
    const unsigned yb = (unsigned)y * (unsigned)sizeof(S);
    Cc f[NPOP];
#pragma unroll
    for (int l = 0; l < NPOP; ++l) f[l] = (Cc)ld_nt(col + (size_t)l * g.ps, yb);
    collide_site<Cc, Store<S>::shifted, WIDE>(f, args);
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_nt(col + (size_t)l * g.ps, yb, (S)f[l]);
    if (WALLS) store_wall_density<S>(f, g, x, y, wall_rho_out);
}

// ---------------------------------------------------------------------------
// Fused step: gather (eq. (4) pull) + wall rule + collide, src -> dst.
//
// On large lattices the FP64 step is launched with FUSED_FP64_LDS_RESERVE
// bytes of dynamic LDS that it does not use: that caps how many of its blocks
// share a CU (2 rather than the 4 its registers allow), so fewer of its
// 74-stream gather/store patterns are in flight at once.  Measured (HIP events,
// median of five runs of 20 launches, two runs each): 2.5-3% faster from
// 1024x2048 to 4096x4096 for any reserve from 56 to 72 KB; no change at
// 1024x1024; 13% slower at 512x512, whose 1024 blocks no longer fit one
// round.  The FP32 step and the other kernels measured slower capped.
// On the largest lattices (from 64 blocks of 256 sites per CU) the FP64 step
// runs 512-thread blocks, one per CU (96 KB reserve): 0.7% faster at
// 2048x4096 and 4096x4096 and 1.2% at 2160x8192, but 3.5% slower at
// 1024x2048 (same A/B, two runs each), so smaller lattices keep the
// 256-thread form.
// ---------------------------------------------------------------------------
constexpr unsigned FUSED_FP64_LDS_RESERVE = 64 * 1024;
// the cap is applied from this many site blocks (of SITE_THREADS) per CU on
constexpr unsigned FUSED_FP64_CAP_MIN_BLOCKS_PER_CU = 16;
constexpr int FUSED_FP64_WIDE_THREADS = 512;
constexpr unsigned FUSED_FP64_WIDE_LDS_RESERVE = 96 * 1024;
constexpr unsigned FUSED_FP64_WIDE_MIN_BLOCKS_PER_CU = 64;

// Launch settings of the FP64 fused step (and of its access-pattern probe)
// for a lattice of nb256 blocks of SITE_THREADS sites on a GPU of ncu CUs
// with max_lds bytes of LDS per block: threads per block and dynamic LDS.
struct FusedLaunch { int threads; unsigned lds; };
inline FusedLaunch fused_fp64_launch(size_t nb256, int ncu, int max_lds)
{
    if (ncu > 0 && nb256 >= (size_t)FUSED_FP64_WIDE_MIN_BLOCKS_PER_CU * (size_t)ncu &&
        (size_t)max_lds >= FUSED_FP64_WIDE_LDS_RESERVE)
        return {FUSED_FP64_WIDE_THREADS, FUSED_FP64_WIDE_LDS_RESERVE};
    if (ncu > 0 && nb256 >= (size_t)FUSED_FP64_CAP_MIN_BLOCKS_PER_CU * (size_t)ncu &&
        (size_t)max_lds >= FUSED_FP64_LDS_RESERVE)
        return {SITE_THREADS, FUSED_FP64_LDS_RESERVE};
    return {SITE_THREADS, 0u};
}
// The in-place collide of the split step takes the same kind of cap on large
// lattices: 2 blocks per CU (64 KB) in FP32 (1-5% faster from 1024x2048 on, in
// both layouts) and, in the columns layout, in FP64 (with the streaming
// stores above, 3-4% faster than 1 block per CU and 1-3% faster than full
// occupancy from 1024x1024 to 4096x4096).  In the planes layout the FP64
// collide ran 3% slower with 96 KB and unchanged with 64 KB, so it keeps full
// occupancy.
// Its blocks keep the XCD renumbering although a collide shares no lines
// between blocks: in hardware order the FP64 columns collide ran 14-18%
// slower at 2048x4096 and 4096x4096.
constexpr unsigned COLLIDE_FP64_LDS_RESERVE = 64 * 1024;
constexpr unsigned COLLIDE_FP32_LDS_RESERVE = 64 * 1024;
// The reverse step with FP64 lambda (256-thread blocks, 3 per CU by its
// registers) takes a reserve that leaves 2 blocks per CU only when that does
// not add a round of blocks: rounds = ceil(blocks / (blocks per CU x CUs)).
// That holds on small lattices alone (up to 4 blocks per CU), e.g. 512x512,
// where it runs 12% faster; wherever the cap adds a round it cost 3-60%
// (sweep from 256x256 to 2048x4096).  With FP32 lambda the reverse step runs
// 64-thread blocks and no cap.
constexpr unsigned ADJ_LDS_RESERVE = 64 * 1024;
constexpr int ADJ_CAP_BLOCKS_PER_CU = 2;
// DEV: the device-scope streaming stores (large lattices) or the plain
// non-temporal ones (below DEV_STORES_MIN_BLOCKS_PER_CU blocks per CU)
template <typename S, bool WRAP, bool WALLS, bool WIDE = true, int T = SITE_THREADS, bool DEV = true>
__global__ __launch_bounds__(T) void k_step_fused(const S* __restrict__ src, S* __restrict__ dst, Geo g,
                                                  CollideArgs args, const double* __restrict__ wall_rho, WallTable wt,
                                                  double* __restrict__ wall_rho_out)
{
    using Cc = typename Store<S>::C;
    const SiteBlock sb = site_block<sizeof(S) == 8, T>(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    const unsigned yb = (unsigned)y * (unsigned)sizeof(S);
    Cc f[NPOP];
    // FP64: the 37 gathers are issued at raised wave priority, so a wave that
    // reaches them is not held behind other waves' collide arithmetic
    // (measured 0.4% on the 2048x4096 step; results are unchanged).
    if constexpr (sizeof(S) == 8) __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        int xs = x - EX[l];
        if (WRAP) xs = wrap_x(xs, g.lx);
        f[l] = (Cc)ld_at(src + (size_t)l * g.ps + g.origin + (long long)xs * g.cs - EY[l], yb);
    }
    if constexpr (sizeof(S) == 8) {
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
    }
    if (WALLS && (y < 3 || y >= g.ly - 3)) {
#pragma unroll
        for (int l = 0; l < NPOP; ++l) {
            if (EY[l] == 0) continue;
            const int wall = EY[l] > 0 ? 0 : 1;
            const int r = wall == 0 ? y : g.ly - 1 - y;       // row counted from the wall
            const int en = wall == 0 ? EY[l] : -EY[l];
            if (en > r) {
                const int xs = wrap_x(x - EX[l], g.lx);
                double v = wt.ew[wall][l] * wall_rho[(wall * 3 + (en - r - 1)) * g.lx + xs];
                if (Store<S>::shifted) v -= W_SHELL[SHELL[l]];
                f[l] = (Cc)v;
            }
        }
    }
    collide_site<Cc, Store<S>::shifted, WIDE>(f, args);
    S* col = dst + g.origin + (long long)x * g.cs;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_stream<DEV>(col + (size_t)l * g.ps, yb, (S)f[l]);
    if (WALLS) store_wall_density<S>(f, g, x, y, wall_rho_out);
}

// ---------------------------------------------------------------------------
// Initial states, read-out, copies.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(SITE_THREADS) void k_init_fields(S* __restrict__ buf, Geo g, const double* __restrict__ rho,
                                                           const double* __restrict__ ux, const double* __restrict__ uy,
                                                           const double* __restrict__ T)
{
    const SiteBlock sb = site_block(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    const long long s = (long long)x * g.ly + y;
    const double r = rho[s], vx = ux[s], vy = uy[s], t = T[s];
    S* p = buf + g.origin + (long long)x * g.cs + y;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) p[(size_t)l * g.ps] = (S)feq_pop<Store<S>::shifted>(l, r, vx, vy, t);
}

struct RtProfile { double t_mid, t_amp, p0, width, y_mid; };

template <typename S>
__global__ __launch_bounds__(SITE_THREADS) void k_init_rt(S* __restrict__ buf, Geo g, const double* __restrict__ P, RtProfile pr)
{
    const SiteBlock sb = site_block(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    const double T0 = pr.t_mid - pr.t_amp * tanh((y - pr.y_mid - P[(long long)x * g.ly + y]) / pr.width);
    const double r0 = pr.p0 / T0;
    S* p = buf + g.origin + (long long)x * g.cs + y;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) p[(size_t)l * g.ps] = (S)feq_pop<Store<S>::shifted>(l, r0, 0.0, 0.0, T0);
}

// rho, u, T of eq. (2) in FP64.  Shifted storage uses the deviation form
// rho = 1 + sum d, T - 1 = (sum (x2 - 2) d) / (2 rho) - u2 / 2.
template <typename S>
__device__ __forceinline__ void site_macros(const S* p, long long plane, double& rho, double& ux, double& uy, double& T)
{
    double f[NPOP];
#pragma unroll
    for (int l = 0; l < NPOP; ++l) f[l] = (double)p[(size_t)l * plane];
    double m0, sx, sy, s2;
    hop_moments<double>(f, m0, sx, sy, s2);
    if (Store<S>::shifted) {
        rho = 1.0 + m0;
        ux = C * sx / rho;
        uy = C * sy / rho;
        T = 1.0 + (C2 * s2 - 2.0 * m0) / (2.0 * rho) - 0.5 * (ux * ux + uy * uy);
    } else {
        rho = m0;
        ux = C * sx / rho;
        uy = C * sy / rho;
        T = 0.5 * (xi2_moment(f) / rho - (ux * ux + uy * uy));
    }
}

template <typename S>
__global__ __launch_bounds__(SITE_THREADS) void k_macros(const S* __restrict__ buf, Geo g, double* __restrict__ rho,
                                                      double* __restrict__ ux, double* __restrict__ uy, double* __restrict__ T)
{
    const SiteBlock sb = site_block(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    double r, vx, vy, t;
    site_macros<S>(buf + g.origin + (long long)x * g.cs + y, g.ps, r, vx, vy, t);
    const long long s = (long long)x * g.ly + y;
    rho[s] = r; ux[s] = vx; uy[s] = vy; T[s] = t;
}

// canonical [37][lx][ly] <-> padded, thread per element
template <typename S, bool TO_CANON>
__global__ __launch_bounds__(256) void k_canon_copy(S* __restrict__ buf, S* __restrict__ canon, Geo g)
{
    const int nyb = (g.ly + 255) / 256;
    const int l = blockIdx.y, x = (int)(blockIdx.x / (unsigned)nyb);
    const int y = (int)(blockIdx.x % (unsigned)nyb) * 256 + threadIdx.x;
    if (y >= g.ly) return;
    const size_t pi = (size_t)l * g.ps + g.origin + (long long)x * g.cs + y;
    const size_t ci = ((size_t)l * g.lx + x) * g.ly + y;
    if (TO_CANON) canon[ci] = buf[pi];
    else buf[pi] = canon[ci];
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: fixed grid, wave shuffles in fixed order,
// LDS across waves, then one block over the partials.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over a block of NT threads (NT a multiple of 64), written to out.
// Block sum of N values per thread into out[0..N) (add: out[k] += sum).
template <int N, int NT>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double* __restrict__ out, bool add = false)
{
    static_assert(NT % 64 == 0, "whole wavefronts");
    __shared__ double red[N][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double s = wave_sum(v[i]);
        if (lane == 0) red[i][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = add ? out[threadIdx.x] + s : s;
    }
}

constexpr int RED_BLOCKS = 1024;

template <typename S>
__global__ __launch_bounds__(256) void k_conservation_partial(const S* __restrict__ buf, Geo g, double* __restrict__ partials)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const long long n = (long long)g.lx * g.ly;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int x = (int)(i / g.ly), y = (int)(i % g.ly);
        const S* p = buf + g.origin + (long long)x * g.cs + y;
        double f[NPOP];
#pragma unroll
        for (int l = 0; l < NPOP; ++l) f[l] = (double)p[(size_t)l * g.ps];
        double m0, sx, sy, s2;
        hop_moments<double>(f, m0, sx, sy, s2);
        acc[0] += Store<S>::shifted ? 1.0 + m0 : m0;
        acc[1] += C * sx;
        acc[2] += C * sy;
        acc[3] += Store<S>::shifted ? 2.0 + C2 * s2 : xi2_moment(f);
    }
    block_sum_store<4, 256>(acc, partials + (size_t)blockIdx.x * 4);
}

// out[k] (+)= sum over nparts of partials[p * N + k]: one block of
// REDUCE_THREADS threads, each with 4 interleaved accumulators, then a fixed
// wave/LDS tree.  The order depends only on nparts, so results are bitwise
// reproducible.  CLEAR: each thread zeroes the partials it read.
constexpr int REDUCE_THREADS = 1024;

template <int N, bool ACCUMULATE, bool CLEAR = false>
__global__ __launch_bounds__(REDUCE_THREADS) void k_reduce_partials(double* __restrict__ partials, int nparts,
                                                                    double* __restrict__ out)
{
    double acc[4][N];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < N; ++k) acc[j][k] = 0.0;
    int p = threadIdx.x;
    for (; p + 3 * REDUCE_THREADS < nparts; p += 4 * REDUCE_THREADS) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                double* q = partials + (size_t)(p + j * REDUCE_THREADS) * N + k;
                acc[j][k] += *q;
                if (CLEAR) *q = 0.0;
            }
    }
    for (int j = 0; p + j * REDUCE_THREADS < nparts; ++j)
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double* q = partials + (size_t)(p + j * REDUCE_THREADS) * N + k;
            acc[j][k] += *q;
            if (CLEAR) *q = 0.0;
        }
    double v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = (acc[0][k] + acc[1][k]) + (acc[2][k] + acc[3][k]);
    __shared__ double red[N][REDUCE_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0) red[k][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double t = 0.0;
        for (int w = 0; w < REDUCE_THREADS / 64; ++w) t += red[threadIdx.x][w];
        out[threadIdx.x] = ACCUMULATE ? out[threadIdx.x] + t : t;
    }
}

}  // namespace lbm
