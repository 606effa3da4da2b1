// lbm_api.hip -- host side of liblbm.so: the C ABI declared in include/lbm.h.
//
// The context keeps only host metadata; every byte of device memory the
// library uses is carved out of the caller's workspace (see plan()).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "lbm.h"
#include "lbm_adjoint.hpp"
#include "lbm_kernels.hpp"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    Geo geo;          // population buffers, storage precision
    Geo lgeo;         // adjoint lambda buffers, FP64
    size_t elem;      // bytes per stored population value
    size_t buf_bytes; // one population buffer
    size_t wall_bytes;// one wall-density table (6 * lx doubles)
    size_t state_bytes; // snapshot: population buffer + its wall densities
    size_t off_buf[2];
    size_t off_wall;  // 2 x 6 * lx doubles (double-buffered wall densities)
    size_t off_part;  // RED_BLOCKS * 4 doubles, then 2 doubles of loss/dtau scratch
    size_t off_lam[2];
    size_t off_apart; // adjoint: one double per collide block
    size_t off_adacc; // adjoint: per-block sums of deferred d/dtau terms
    size_t total;
};

Geo make_geo(int lx, int ly, size_t elem, int layout) { return padded_geo(lx, ly, elem, layout == LBM_LAYOUT_PLANES); }

bool valid(const lbm_params* p)
{
    if (!p) return false;
    if (p->lx < 7 || p->ly < 7) return false;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau) || !std::isfinite(p->g_y)) return false;
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32_SHIFTED && p->precision != LBM_FP32_SHIFTED_F32SUMS)
        return false;
    if (p->ybc != LBM_Y_WALLS && p->ybc != LBM_Y_PERIODIC) return false;
    if (p->xmode != LBM_X_WRAP && p->xmode != LBM_X_HALO) return false;
    if (p->step_kind != LBM_STEP_SPLIT && p->step_kind != LBM_STEP_FUSED) return false;
    if (p->layout != LBM_LAYOUT_PLANES && p->layout != LBM_LAYOUT_COLUMNS) return false;
    if (p->adjoint < 0 || p->adjoint > 2) return false;
    if ((long long)p->lx * p->ly > (1LL << 31)) return false;
    return true;
}

Plan plan(const lbm_params* p)
{
    Plan pl{};
    pl.elem = p->precision == LBM_FP64 ? 8 : 4;
    pl.geo = make_geo(p->lx, p->ly, pl.elem, p->layout);
    pl.lgeo = make_geo(p->lx, p->ly, p->adjoint == 2 ? 4 : 8, p->layout);
    pl.buf_bytes = align_up((size_t)pl.geo.total * pl.elem, ALIGN);
    pl.wall_bytes = align_up(6 * (size_t)p->lx * 8, ALIGN);
    pl.state_bytes = pl.buf_bytes + pl.wall_bytes;
    size_t off = 0;
    pl.off_buf[0] = off; off += pl.buf_bytes;
    pl.off_buf[1] = off; off += pl.buf_bytes;
    pl.off_wall = off; off += 2 * pl.wall_bytes;
    pl.off_part = off; off += align_up(((size_t)RED_BLOCKS * 4 + 2) * 8, ALIGN);
    if (p->adjoint) {
        const size_t lb = align_up((size_t)pl.lgeo.total * (p->adjoint == 2 ? 4 : 8), ALIGN);
        pl.off_lam[0] = off; off += lb;
        pl.off_lam[1] = off; off += lb;
        // one partial per block of the reverse step (its blocks are the
        // smallest of the adjoint launches)
        const int at = p->adjoint == 2 ? adj_threads<float>() : adj_threads<double>();
        const size_t nb = (size_t)((p->ly + at - 1) / at) * p->lx;
        pl.off_apart = off; off += align_up(nb * 8, ALIGN);
        pl.off_adacc = off; off += align_up(nb * 8, ALIGN);
    }
    pl.total = off;
    return pl;
}

thread_local std::string g_create_error;

}  // namespace

struct lbm_ctx {
    lbm_params p;
    Plan pl;
    char* ws;
    hipStream_t stream;
    int cur;           // current population buffer
    bool have_prev;    // the other buffer holds the state before the last propagate
    int lam_cur;
    bool have_lambda;
    // lambda buffer lam_cur holds mu of the last reverse step (lambda is its
    // propagate^T + bc^T gather) rather than lambda itself
    bool lam_is_mu;
    // wall densities (rows 0..2 and ly-3..ly-1) of population buffer wr_buf
    // (-1: none) live in wall table wr_cur; the other table receives the
    // densities the next collide or fused step writes
    int wr_cur;
    int wr_buf;
    WallTable wt;
    CollideArgs cargs;
    unsigned fused_lds;  // dynamic LDS of the fused step's launch (occupancy cap; 0: none)
    int fused_threads;   // threads per block of the FP64 fused step (256 or 512)
    unsigned collide_lds;// the same for the split step's collide
    bool dev_stores;     // fused and reverse steps with device-scope stores (dev_stores_for)
    unsigned adj_lds;    // the same for the reverse step
    std::string err;

    void* buf(int i) { return ws + pl.off_buf[i]; }
    double* wall_rho(int i) { return reinterpret_cast<double*>(ws + pl.off_wall + i * pl.wall_bytes); }
    double* partials() { return reinterpret_cast<double*>(ws + pl.off_part); }
    double* scratch2() { return partials() + (size_t)RED_BLOCKS * 4; }
    template <typename L> L* lam(int i) { return reinterpret_cast<L*>(ws + pl.off_lam[i]); }
    bool fp64() const { return p.precision == LBM_FP64; }
    bool f32_sums() const { return p.precision == LBM_FP32_SHIFTED_F32SUMS; }
    bool lam32() const { return p.adjoint == 2; }
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const char* what)
{
    c->err = what;
    return s;
}

lbm_status check_launch(lbm_ctx* c, const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string(what) + ": " + hipGetErrorString(e);
        return LBM_ERR_HIP;
    }
    return LBM_OK;
}

void set_collide_args(lbm_ctx* c)
{
    const double tau = c->p.tau, g = c->p.g_y;
    c->cargs.omega = 1.0 / tau;
    c->cargs.tau_g = tau * g;
    c->cargs.grav_th = tau * (1.0 - tau) * g * g / 2.0;
    c->cargs.g = g;
    c->cargs.g_f = (float)g;
    c->cargs.omega_f = (float)c->cargs.omega;
    c->cargs.tau_g_f = (float)c->cargs.tau_g;
    c->cargs.grav_th_f = (float)c->cargs.grav_th;
}

// 1-D grid of site blocks, renumbered per XCD inside the kernels (site_block)
dim3 site_grid(const Geo& g) { return dim3((unsigned)((g.ly + SITE_THREADS - 1) / SITE_THREADS) * (unsigned)g.lx); }

template <typename S>
lbm_status launch_propagate(lbm_ctx* c, const S* src, S* dst)
{
    const Geo& g = c->pl.geo;
    constexpr int VEC = sizeof(S) == 8 ? 2 : 4;
    constexpr int UNROLL = PROP_UNROLL;
    constexpr int CH = PROP_THREADS * VEC * UNROLL;
    const size_t nch = (size_t)((g.ly + CH - 1) / CH);
    const size_t nblk = nch * NPOP * (size_t)g.lx;
    if (nblk > 0xffffffffull) return fail(c, LBM_ERR_SIZE, "propagate: lattice too large for one grid");
    const unsigned gx = nblk < PROP_GRID_X ? (unsigned)nblk : PROP_GRID_X;
    const dim3 grid(gx, (unsigned)((nblk + gx - 1) / gx));
    const bool cols = c->p.layout == LBM_LAYOUT_COLUMNS;
    const bool wrap = c->p.xmode == LBM_X_WRAP;
    const unsigned nb = (unsigned)nblk;
    if (wrap && cols)
        hipLaunchKernelGGL((k_propagate<S, VEC, UNROLL, true, true>), grid, dim3(PROP_THREADS), 0, c->stream, src, dst, g, nb);
    else if (wrap)
        hipLaunchKernelGGL((k_propagate<S, VEC, UNROLL, true, false>), grid, dim3(PROP_THREADS), 0, c->stream, src, dst, g, nb);
    else if (cols)
        hipLaunchKernelGGL((k_propagate<S, VEC, UNROLL, false, true>), grid, dim3(PROP_THREADS), 0, c->stream, src, dst, g, nb);
    else
        hipLaunchKernelGGL((k_propagate<S, VEC, UNROLL, false, false>), grid, dim3(PROP_THREADS), 0, c->stream, src, dst, g, nb);
    return check_launch(c, "propagate");
}

template <typename S>
lbm_status launch_pre_stream(lbm_ctx* c, S* src)
{
    // halos the pull of the current buffer needs: y ghost rows if periodic,
    // then x halo columns (whole padded columns, so corners follow).
    const Geo& g = c->pl.geo;
    if (c->p.ybc == LBM_Y_PERIODIC) {
        dim3 grid((g.lx * 6 + 255) / 256, NPOP);
        hipLaunchKernelGGL((k_fill_y_ghosts<S>), grid, dim3(256), 0, c->stream, src, g);
        lbm_status s = check_launch(c, "fill_y_ghosts");
        if (s) return s;
    }
    if (c->p.xmode == LBM_X_HALO) {
        dim3 grid((g.lyp + 255) / 256, 3, NPOP);
        hipLaunchKernelGGL((k_fill_x_halo<S>), grid, dim3(256), 0, c->stream, src, g);
        lbm_status s = check_launch(c, "fill_x_halo");
        if (s) return s;
    }
    return LBM_OK;
}

template <typename S>
lbm_status launch_wall_density(lbm_ctx* c, const S* src, double* out)
{
    const Geo& g = c->pl.geo;
    hipLaunchKernelGGL((k_wall_density<S>), dim3((6 * g.lx + 255) / 256), dim3(256), 0, c->stream, src, g, out);
    return check_launch(c, "wall_density");
}

// Makes wall table wr_cur hold the wall densities of population buffer b.
template <typename S>
lbm_status ensure_wall_density(lbm_ctx* c, int b)
{
    if (c->wr_buf == b) return LBM_OK;
    lbm_status s = launch_wall_density<S>(c, (const S*)c->buf(b), c->wall_rho(c->wr_cur));
    if (s) return s;
    c->wr_buf = b;
    return LBM_OK;
}

template <typename S>
lbm_status do_propagate(lbm_ctx* c)
{
    S* src = (S*)c->buf(c->cur);
    S* dst = (S*)c->buf(1 - c->cur);
    lbm_status s = launch_pre_stream<S>(c, src);
    if (s) return s;
    s = launch_propagate<S>(c, src, dst);
    if (s) return s;
    if (c->wr_buf == 1 - c->cur) c->wr_buf = -1;   // destination overwritten
    c->cur = 1 - c->cur;
    c->have_prev = true;
    return LBM_OK;
}

template <typename S>
lbm_status do_bc(lbm_ctx* c)
{
    if (c->p.ybc == LBM_Y_PERIODIC) return LBM_OK;
    if (!c->have_prev) return fail(c, LBM_ERR_STATE, "bc: no propagate since the state was set");
    const Geo& g = c->pl.geo;
    lbm_status s = ensure_wall_density<S>(c, 1 - c->cur);
    if (s) return s;
    hipLaunchKernelGGL((k_bc_apply<S>), dim3((NSLOT * g.lx + 255) / 256), dim3(256), 0, c->stream,
                       (S*)c->buf(c->cur), g, (const double*)c->wall_rho(c->wr_cur), c->wt);
    return check_launch(c, "bc_apply");
}

// In-place collide of the current buffer; wo receives the wall densities
// (WALLS) -- FP32 storage with FP32 sums takes the WIDE = false kernels.
template <typename S, bool WALLS>
void launch_collide(lbm_ctx* c, double* wo)
{
    const Geo& g = c->pl.geo;
    if constexpr (std::is_same<S, float>::value) {
        if (c->f32_sums()) {
            hipLaunchKernelGGL((k_collide<S, WALLS, false>), site_grid(g), dim3(SITE_THREADS), c->collide_lds,
                               c->stream, (S*)c->buf(c->cur), g, c->cargs, wo);
            return;
        }
    }
    hipLaunchKernelGGL((k_collide<S, WALLS, true>), site_grid(g), dim3(SITE_THREADS), c->collide_lds, c->stream,
                       (S*)c->buf(c->cur), g, c->cargs, wo);
}

template <typename S>
lbm_status do_collide(lbm_ctx* c)
{
    if (c->p.ybc == LBM_Y_WALLS) {
        launch_collide<S, true>(c, c->wall_rho(1 - c->wr_cur));
        lbm_status s = check_launch(c, "collide");
        if (s) return s;
        c->wr_cur = 1 - c->wr_cur;
        c->wr_buf = c->cur;
        return LBM_OK;
    }
    launch_collide<S, false>(c, (double*)nullptr);
    return check_launch(c, "collide");
}

// One fused step src -> dst (wall densities read from wr, written to wo),
// T threads per block.
template <typename S, bool WIDE, int T, bool DEV>
void launch_fused_kernel_dev(lbm_ctx* c, const S* src, S* dst, const double* wr, double* wo)
{
    const Geo& g = c->pl.geo;
    const bool walls = c->p.ybc == LBM_Y_WALLS;
    const bool wrap = c->p.xmode == LBM_X_WRAP;
    const unsigned lds = sizeof(S) == 8 ? c->fused_lds : 0u;
    const dim3 grid((unsigned)((g.ly + T - 1) / T) * (unsigned)g.lx);
    if (wrap && walls)
        hipLaunchKernelGGL((k_step_fused<S, true, true, WIDE, T, DEV>), grid, dim3(T), lds, c->stream, src, dst, g,
                           c->cargs, wr, c->wt, wo);
    else if (wrap)
        hipLaunchKernelGGL((k_step_fused<S, true, false, WIDE, T, DEV>), grid, dim3(T), lds, c->stream, src, dst, g,
                           c->cargs, wr, c->wt, wo);
    else if (walls)
        hipLaunchKernelGGL((k_step_fused<S, false, true, WIDE, T, DEV>), grid, dim3(T), lds, c->stream, src, dst, g,
                           c->cargs, wr, c->wt, wo);
    else
        hipLaunchKernelGGL((k_step_fused<S, false, false, WIDE, T, DEV>), grid, dim3(T), lds, c->stream, src, dst, g,
                           c->cargs, wr, c->wt, wo);
}
template <typename S, bool WIDE, int T>
void launch_fused_kernel(lbm_ctx* c, const S* src, S* dst, const double* wr, double* wo)
{
    if (c->dev_stores) launch_fused_kernel_dev<S, WIDE, T, true>(c, src, dst, wr, wo);
    else launch_fused_kernel_dev<S, WIDE, T, false>(c, src, dst, wr, wo);
}

template <typename S>
void launch_fused(lbm_ctx* c, const S* src, S* dst, const double* wr, double* wo)
{
    if constexpr (std::is_same<S, float>::value) {
        if (c->f32_sums()) {
            launch_fused_kernel<S, false, SITE_THREADS>(c, src, dst, wr, wo);
            return;
        }
        launch_fused_kernel<S, true, SITE_THREADS>(c, src, dst, wr, wo);
    } else {
        if (c->fused_threads == FUSED_FP64_WIDE_THREADS)
            launch_fused_kernel<S, true, FUSED_FP64_WIDE_THREADS>(c, src, dst, wr, wo);
        else
            launch_fused_kernel<S, true, SITE_THREADS>(c, src, dst, wr, wo);
    }
}

template <typename S>
lbm_status do_step_fused(lbm_ctx* c)
{
    S* src = (S*)c->buf(c->cur);
    S* dst = (S*)c->buf(1 - c->cur);
    lbm_status s = launch_pre_stream<S>(c, src);
    if (s) return s;
    const bool walls = c->p.ybc == LBM_Y_WALLS;
    if (walls) {
        s = ensure_wall_density<S>(c, c->cur);
        if (s) return s;
    }
    launch_fused<S>(c, src, dst, c->wall_rho(c->wr_cur), c->wall_rho(1 - c->wr_cur));
    s = check_launch(c, "step_fused");
    if (s) return s;
    c->cur = 1 - c->cur;
    c->have_prev = true;
    if (walls) {
        c->wr_cur = 1 - c->wr_cur;
        c->wr_buf = c->cur;
    }
    return LBM_OK;
}

template <typename S>
lbm_status do_step(lbm_ctx* c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        lbm_status s;
        if (c->p.step_kind == LBM_STEP_FUSED) {
            s = do_step_fused<S>(c);
        } else {
            s = do_propagate<S>(c);
            if (!s) s = do_bc<S>(c);
            if (!s) s = do_collide<S>(c);
        }
        if (s) return s;
    }
    return LBM_OK;
}

#define DISPATCH(c, fn, ...) ((c)->fp64() ? fn<double>(c, ##__VA_ARGS__) : fn<float>(c, ##__VA_ARGS__))
// storage type S and adjoint-state type L
#define ADJ_DISPATCH(c, fn, ...)                                                                \
    ((c)->fp64() ? ((c)->lam32() ? fn<double, float>(c, ##__VA_ARGS__) : fn<double, double>(c, ##__VA_ARGS__)) \
                 : ((c)->lam32() ? fn<float, float>(c, ##__VA_ARGS__) : fn<float, double>(c, ##__VA_ARGS__)))
#define LAM_DISPATCH(c, fn, ...) ((c)->lam32() ? fn<float>(c, ##__VA_ARGS__) : fn<double>(c, ##__VA_ARGS__))

template <typename S>
lbm_status do_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T)
{
    hipLaunchKernelGGL((k_init_fields<S>), site_grid(c->pl.geo), dim3(SITE_THREADS), 0, c->stream,
                       (S*)c->buf(c->cur), c->pl.geo, rho, ux, uy, T);
    c->have_prev = false;
    c->wr_buf = -1;
    return check_launch(c, "init");
}
template <typename S>
lbm_status do_init_rt(lbm_ctx* c, const double* P, RtProfile pr)
{
    hipLaunchKernelGGL((k_init_rt<S>), site_grid(c->pl.geo), dim3(SITE_THREADS), 0, c->stream,
                       (S*)c->buf(c->cur), c->pl.geo, P, pr);
    c->have_prev = false;
    c->wr_buf = -1;
    return check_launch(c, "init_rt");
}
template <typename S>
lbm_status do_macros(lbm_ctx* c, double* rho, double* ux, double* uy, double* T)
{
    hipLaunchKernelGGL((k_macros<S>), site_grid(c->pl.geo), dim3(SITE_THREADS), 0, c->stream,
                       (const S*)c->buf(c->cur), c->pl.geo, rho, ux, uy, T);
    return check_launch(c, "macros");
}
template <typename S>
lbm_status do_canon(lbm_ctx* c, void* canon, bool to_canon)
{
    const Geo& g = c->pl.geo;
    dim3 grid((unsigned)((g.ly + 255) / 256) * (unsigned)g.lx, NPOP);
    if (to_canon)
        hipLaunchKernelGGL((k_canon_copy<S, true>), grid, dim3(256), 0, c->stream, (S*)c->buf(c->cur), (S*)canon, g);
    else
        hipLaunchKernelGGL((k_canon_copy<S, false>), grid, dim3(256), 0, c->stream, (S*)c->buf(c->cur), (S*)canon, g);
    if (!to_canon) {
        c->have_prev = false;
        c->wr_buf = -1;
    }
    return check_launch(c, "canonical copy");
}
// snapshot = current population buffer + its wall densities (walls only)
template <typename S>
lbm_status do_get_state(lbm_ctx* c, char* dst)
{
    if (hipMemcpyAsync(dst, c->buf(c->cur), c->pl.buf_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return check_launch(c, "get_state");
    if (c->p.ybc == LBM_Y_WALLS) {
        lbm_status s = ensure_wall_density<S>(c, c->cur);
        if (s) return s;
        if (hipMemcpyAsync(dst + c->pl.buf_bytes, c->wall_rho(c->wr_cur), c->pl.wall_bytes, hipMemcpyDeviceToDevice,
                           c->stream) != hipSuccess)
            return check_launch(c, "get_state");
    }
    return LBM_OK;
}

// One fused step from snapshot src into snapshot dst (both buffer + wall
// densities); the context's own buffers and wall tables are not touched.
template <typename S>
lbm_status do_step_state(lbm_ctx* c, char* src, char* dst)
{
    S* sb = (S*)src;
    S* db = (S*)dst;
    lbm_status s = launch_pre_stream<S>(c, sb);   // padding of the source only
    if (s) return s;
    const bool walls = c->p.ybc == LBM_Y_WALLS;
    const double* wr = walls ? (const double*)(src + c->pl.buf_bytes) : nullptr;
    double* wo = walls ? (double*)(dst + c->pl.buf_bytes) : nullptr;
    launch_fused<S>(c, sb, db, wr, wo);
    return check_launch(c, "step_state");
}

template <typename S>
lbm_status do_conservation(lbm_ctx* c, double* out4)
{
    hipLaunchKernelGGL((k_conservation_partial<S>), dim3(RED_BLOCKS), dim3(256), 0, c->stream,
                       (const S*)c->buf(c->cur), c->pl.geo, c->partials());
    lbm_status s = check_launch(c, "conservation");
    if (s) return s;
    hipLaunchKernelGGL((k_reduce_partials<4, false>), dim3(1), dim3(REDUCE_THREADS), 0, c->stream,
                       c->partials(), RED_BLOCKS, out4);
    return check_launch(c, "conservation reduce");
}
}  // namespace

// ----------------------------------------------------------------------------
// Scratch of lbm_conservation_noalloc: the reduction's block partials
// (RED_BLOCKS x 4 doubles, 32 KiB) in a fixed device array instead of a
// workspace.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (that device current) and only that address reaches
// kernels.  Every call on one device shares the array.
// ----------------------------------------------------------------------------
static __device__ __align__(256) double scratch[RED_BLOCKS * 4];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES];   // device address of `scratch`, per device

// Device address of `scratch` on the current device (looked up on the first
// call there).
lbm_status scratch_on_current_device(double** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        g_create_error = "conservation_noalloc: no usable current device";
        return LBM_ERR_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_create_error = std::string("conservation_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e);
            return LBM_ERR_HIP;
        }
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

// Geometry of a canonical [37][lx][ly] array: no padding, no halos.
Geo canonical_geo(int lx, int ly)
{
    Geo g{};
    g.lx = lx;
    g.ly = ly;
    g.lyp = ly;
    g.g = 0;
    g.cs = ly;
    g.ps = (long long)lx * ly;
    g.origin = 0;
    g.total = NPOP * g.ps;
    return g;
}

template <typename S>
lbm_status launch_conservation_noalloc(const Geo& g, const void* pops, double* part, double* out4, hipStream_t st)
{
    hipLaunchKernelGGL((k_conservation_partial<S>), dim3(RED_BLOCKS), dim3(256), 0, st, (const S*)pops, g, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL((k_reduce_partials<4, false>), dim3(1), dim3(REDUCE_THREADS), 0, st,
                           part, RED_BLOCKS, out4);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        g_create_error = std::string("conservation_noalloc: ") + hipGetErrorString(e);
        return LBM_ERR_HIP;
    }
    return LBM_OK;
}

}  // namespace

namespace {

// Blocks of the reverse step's kernel that fit one CU at full occupancy
// (0 if the runtime cannot tell).
template <typename S, typename L>
int adj_blocks_per_cu_t(bool dev_stores)
{
    int n = 0;
    constexpr int T = adj_threads<L>();
    const hipError_t e =
        dev_stores ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adj_collide<S, L, true, true, T, true>, T, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adj_collide<S, L, true, true, T, false>, T, 0);
    return e == hipSuccess ? n : 0;
}

// blocks per CU of the reverse step this context launches
int adj_blocks_per_cu(const lbm_params* p, bool dev_stores)
{
    const bool lam32 = p->adjoint == 2;
    if (p->precision == LBM_FP64)
        return lam32 ? adj_blocks_per_cu_t<double, float>(dev_stores) : adj_blocks_per_cu_t<double, double>(dev_stores);
    return lam32 ? adj_blocks_per_cu_t<float, float>(dev_stores) : adj_blocks_per_cu_t<float, double>(dev_stores);
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) { return valid(p) ? plan(p).total : 0; }

size_t lbm_state_bytes(const lbm_params* p) { return valid(p) ? plan(p).state_bytes : 0; }

lbm_status lbm_create(const lbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream, lbm_ctx** out)
{
    if (!out) { g_create_error = "out is NULL"; return LBM_ERR_INVALID; }
    *out = nullptr;
    if (!valid(p)) { g_create_error = "invalid parameters"; return LBM_ERR_INVALID; }
    Plan pl = plan(p);
    if (!dev_workspace) { g_create_error = "workspace is NULL"; return LBM_ERR_INVALID; }
    if ((uintptr_t)dev_workspace % ALIGN) { g_create_error = "workspace not 256-byte aligned"; return LBM_ERR_INVALID; }
    if (bytes < pl.total) { g_create_error = "workspace too small"; return LBM_ERR_SIZE; }
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    c->pl = pl;
    c->ws = (char*)dev_workspace;
    c->stream = (hipStream_t)hip_stream;
    c->cur = 0;
    c->have_prev = false;
    c->lam_cur = 0;
    c->have_lambda = false;
    c->lam_is_mu = false;
    c->wr_cur = 0;
    c->wr_buf = -1;
    for (int l = 0; l < NPOP; ++l) {
        c->wt.ew[0][l] = feq_pop<false>(l, 1.0, 0.0, 0.0, p->t_bottom);
        c->wt.ew[1][l] = feq_pop<false>(l, 1.0, 0.0, 0.0, p->t_top);
        c->wt.w[l] = W_SHELL[SHELL[l]];
    }
    set_collide_args(c);
    // occupancy caps of the FP64 fused step and of the collide on large
    // lattices (lbm_kernels.hpp)
    c->fused_lds = 0;
    c->fused_threads = SITE_THREADS;
    c->collide_lds = 0;
    c->dev_stores = false;
    int dev = 0, ncu = 0, max_lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && ncu > 0) {
        const FusedLaunch fl = fused_fp64_launch(site_grid(pl.geo).x, ncu, max_lds);
        c->fused_threads = fl.threads;
        c->fused_lds = fl.lds;
        c->dev_stores = dev_stores_for(site_grid(pl.geo).x, ncu);
        if ((size_t)site_grid(pl.geo).x >= (size_t)FUSED_FP64_CAP_MIN_BLOCKS_PER_CU * (size_t)ncu) {
            const unsigned coll = p->precision == LBM_FP64 ? COLLIDE_FP64_LDS_RESERVE : COLLIDE_FP32_LDS_RESERVE;
            if ((size_t)max_lds >= coll && (p->precision != LBM_FP64 || p->layout == LBM_LAYOUT_COLUMNS))
                c->collide_lds = coll;
        }
    }
    c->adj_lds = 0;
    // (256-thread reverse steps only: FP64 lambda)
    if (p->adjoint == 1 && ncu > 0 && (size_t)max_lds >= ADJ_LDS_RESERVE) {
        const int full = adj_blocks_per_cu(p, c->dev_stores);
        const size_t nb = site_grid(pl.geo).x;
        auto rounds = [&](int per_cu) { return (nb + (size_t)per_cu * ncu - 1) / ((size_t)per_cu * ncu); };
        if (full > ADJ_CAP_BLOCKS_PER_CU && rounds(ADJ_CAP_BLOCKS_PER_CU) <= rounds(full))
            c->adj_lds = ADJ_LDS_RESERVE;
    }
    if (hipMemsetAsync(dev_workspace, 0, pl.total, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        g_create_error = "workspace initialisation failed";
        delete c;
        return LBM_ERR_HIP;
    }
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) { delete ctx; }

lbm_status lbm_set_tau(lbm_ctx* c, double tau)
{
    if (!c) return LBM_ERR_INVALID;
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(c, LBM_ERR_INVALID, "tau must be > 0.5");
    c->p.tau = tau;
    set_collide_args(c);
    return LBM_OK;
}


lbm_status lbm_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T)
{
    if (!c) return LBM_ERR_INVALID;
    if (!rho || !ux || !uy || !T) return fail(c, LBM_ERR_INVALID, "init: NULL field");
    return DISPATCH(c, do_init, rho, ux, uy, T);
}

lbm_status lbm_init_rt(lbm_ctx* c, const double* P, const lbm_rt_profile* prof)
{
    if (!c) return LBM_ERR_INVALID;
    if (!P || !prof) return fail(c, LBM_ERR_INVALID, "init_rt: NULL argument");
    if (!(prof->width > 0.0) || !(prof->p0 > 0.0)) return fail(c, LBM_ERR_INVALID, "init_rt: width and p0 must be > 0");
    RtProfile pr{prof->t_mid, prof->t_amp, prof->p0, prof->width, prof->y_mid};
    return DISPATCH(c, do_init_rt, P, pr);
}

lbm_status lbm_propagate(lbm_ctx* c)
{
    if (!c) return LBM_ERR_INVALID;
    return DISPATCH(c, do_propagate);
}

lbm_status lbm_bc(lbm_ctx* c)
{
    if (!c) return LBM_ERR_INVALID;
    return DISPATCH(c, do_bc);
}

lbm_status lbm_collide(lbm_ctx* c)
{
    if (!c) return LBM_ERR_INVALID;
    return DISPATCH(c, do_collide);
}

lbm_status lbm_step(lbm_ctx* c, int64_t n)
{
    if (!c) return LBM_ERR_INVALID;
    if (n < 0) return fail(c, LBM_ERR_INVALID, "step: n < 0");
    return DISPATCH(c, do_step, n);
}

lbm_status lbm_get_macros(lbm_ctx* c, double* rho, double* ux, double* uy, double* T)
{
    if (!c) return LBM_ERR_INVALID;
    if (!rho || !ux || !uy || !T) return fail(c, LBM_ERR_INVALID, "get_macros: NULL field");
    return DISPATCH(c, do_macros, rho, ux, uy, T);
}

lbm_status lbm_get_pops(lbm_ctx* c, void* dst)
{
    if (!c) return LBM_ERR_INVALID;
    if (!dst) return fail(c, LBM_ERR_INVALID, "get_pops: NULL");
    return DISPATCH(c, do_canon, dst, true);
}

lbm_status lbm_set_pops(lbm_ctx* c, const void* src)
{
    if (!c) return LBM_ERR_INVALID;
    if (!src) return fail(c, LBM_ERR_INVALID, "set_pops: NULL");
    return DISPATCH(c, do_canon, const_cast<void*>(src), false);
}

lbm_status lbm_get_state(lbm_ctx* c, void* dst)
{
    if (!c) return LBM_ERR_INVALID;
    if (!dst) return fail(c, LBM_ERR_INVALID, "get_state: NULL");
    return DISPATCH(c, do_get_state, (char*)dst);
}

lbm_status lbm_set_state(lbm_ctx* c, const void* src)
{
    if (!c) return LBM_ERR_INVALID;
    if (!src) return fail(c, LBM_ERR_INVALID, "set_state: NULL");
    const char* s = (const char*)src;
    if (hipMemcpyAsync(c->buf(c->cur), s, c->pl.buf_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return check_launch(c, "set_state");
    c->have_prev = false;
    c->wr_buf = -1;
    if (c->p.ybc == LBM_Y_WALLS) {
        if (hipMemcpyAsync(c->wall_rho(c->wr_cur), s + c->pl.buf_bytes, c->pl.wall_bytes, hipMemcpyDeviceToDevice,
                           c->stream) != hipSuccess)
            return check_launch(c, "set_state");
        c->wr_buf = c->cur;
    }
    return LBM_OK;
}

lbm_status lbm_step_state(lbm_ctx* c, void* src_state, void* dst_state)
{
    if (!c) return LBM_ERR_INVALID;
    if (!src_state || !dst_state) return fail(c, LBM_ERR_INVALID, "step_state: NULL");
    if (((uintptr_t)src_state | (uintptr_t)dst_state) % ALIGN != 0)
        return fail(c, LBM_ERR_INVALID, "step_state: snapshots must be 256-byte aligned");
    const char* a = (const char*)src_state;
    const char* b = (const char*)dst_state;
    const size_t n = c->pl.state_bytes;
    if (a < b + n && b < a + n) return fail(c, LBM_ERR_INVALID, "step_state: snapshots overlap");
    return DISPATCH(c, do_step_state, (char*)src_state, (char*)dst_state);
}

lbm_status lbm_conservation(lbm_ctx* c, double* dev_out4)
{
    if (!c) return LBM_ERR_INVALID;
    if (!dev_out4) return fail(c, LBM_ERR_INVALID, "conservation: NULL");
    return DISPATCH(c, do_conservation, dev_out4);
}

lbm_status lbm_conservation_noalloc(int precision, int lx, int ly, const void* pops, double* dev_out4,
                                    void* hip_stream)
{
    if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED && precision != LBM_FP32_SHIFTED_F32SUMS) {
        g_create_error = "conservation_noalloc: unknown precision";
        return LBM_ERR_INVALID;
    }
    if (lx < 1 || ly < 1) {
        g_create_error = "conservation_noalloc: lx and ly must be >= 1";
        return LBM_ERR_INVALID;
    }
    if ((long long)lx * ly > LBM_NOALLOC_MAX_SITES) {
        g_create_error = "conservation_noalloc: lattice exceeds LBM_NOALLOC_MAX_SITES (2^31) sites";
        return LBM_ERR_SIZE;
    }
    if (!pops || !dev_out4) {
        g_create_error = "conservation_noalloc: NULL pointer";
        return LBM_ERR_INVALID;
    }
    double* part = nullptr;
    lbm_status s = scratch_on_current_device(&part);
    if (s) return s;
    const Geo g = canonical_geo(lx, ly);
    const hipStream_t st = (hipStream_t)hip_stream;
    return precision == LBM_FP64 ? launch_conservation_noalloc<double>(g, pops, part, dev_out4, st)
                                 : launch_conservation_noalloc<float>(g, pops, part, dev_out4, st);
}

lbm_status lbm_sync(lbm_ctx* c)
{
    if (!c) return LBM_ERR_INVALID;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->err = std::string("sync: ") + hipGetErrorString(e);
        return LBM_ERR_HIP;
    }
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void lbm_velocity_table(int8_t ex[LBM_NPOP], int8_t ey[LBM_NPOP])
{
    for (int l = 0; l < NPOP; ++l) { ex[l] = (int8_t)EX[l]; ey[l] = (int8_t)EY[l]; }
}

void lbm_weights(double w[LBM_NPOP])
{
    for (int l = 0; l < NPOP; ++l) w[l] = W_SHELL[SHELL[l]];
}

double lbm_scale_c(void) { return C; }

}  // extern "C"

#include "lbm_adjoint_api.inc"
#include "lbm_layouts_api.inc"
#include "lbm_hetero_api.inc"
