// copy_probe.hip -- reference streaming copy for roofline calibration.
//
// Not part of the lattice Boltzmann path: the benchmark times it beside
// propagate, on a buffer the size of one population buffer, so that
// propagate's bandwidth can be quoted as a fraction of a plain copy measured
// on the same GPU in the same run.  dst[i] = src[i] over `bytes` bytes in
// 16-byte vectors, one workgroup per chunk of `block_bytes` bytes (1024, 2048
// or 4096: 64, 128 or 256 threads), non-temporal loads and the library's
// streaming stores (non-temporal, device scope: lbm::st_nt), hardware block
// order (the fastest plain copy measured on MI355X used this form).
//
// int cp_copy(const void* src, void* dst, size_t bytes, int block_bytes,
//             void* hip_stream)
//   src, dst: device pointers, 16-byte aligned, not overlapping; bytes a
//   multiple of 16.  Enqueued on hip_stream (a hipStream_t, 0 = default
//   stream); returns without waiting.  Returns 0 on success, 1 for an invalid
//   argument (nothing launched), 2 if the launch failed.
//
// The second probe is the fused step's own memory access pattern with no
// arithmetic: on a padded columns-layout buffer of the library (the geometry
// of lbm_kernels.hpp), every site gathers its 37 populations from
// (x - e_x mod lx, y - e_y) and stores them at its own site, with the same
// workgroups (block size and, FP64 on large lattices, occupancy cap), block
// renumbering, load priority and store form as the FP64 / FP32 fused step
// (walls and the collision left out).  It is the streaming of eq. (4) evaluated per site, so
// dst equals a propagate of src.  Its time is the ceiling that access pattern
// leaves the fused step.
//
// The third probe is the reverse step's access pattern over FP32 states: per
// site, 37 populations gathered from (x - e_x, y - e_y) of an FP32 state
// buffer, 37 gathered from (x + e_x, y + e_y) of a lambda buffer (FP32 or
// FP64), and mu_l = f_l + lambda_l stored at the site, with the reverse
// step's workgroups (64 threads with FP32 lambda, 256 with FP64) and block
// renumbering (the collide^T arithmetic and the wall terms left out).
//
// size_t cp_gather_bytes(int elem_bytes, int lx, int ly)
//   bytes of one buffer (elem_bytes 8 or 4; lx, ly >= 7; lx ly <= 2^31),
//   0 if invalid.
// int cp_gather_copy(int elem_bytes, int lx, int ly, const void* src,
//                    void* dst, void* hip_stream)
//   src, dst: distinct device buffers of cp_gather_bytes bytes, 256-byte
//   aligned.  Returns as cp_copy.
// int cp_adjoint_pattern(int lam_bytes, int lx, int ly, const void* f,
//                        const void* lam, void* mu, void* hip_stream)
//   f: cp_gather_bytes(4, lx, ly) bytes; lam, mu: cp_gather_bytes(lam_bytes,
//   lx, ly) bytes each (lam_bytes 4 or 8); three distinct 256-byte aligned
//   device buffers.  Returns as cp_copy.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm_adjoint.hpp"
#include "lbm_kernels.hpp"

namespace {

template <typename S, int T = lbm::SITE_THREADS>
__global__ __launch_bounds__(T) void k_gather_copy(const S* __restrict__ src, S* __restrict__ dst, lbm::Geo g)
{
    using namespace lbm;
    const SiteBlock sb = site_block<sizeof(S) == 8, T>(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    const unsigned yb = (unsigned)y * (unsigned)sizeof(S);
    S f[NPOP];
    if constexpr (sizeof(S) == 8) __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        const int xs = wrap_x(x - EX[l], g.lx);
        f[l] = ld_at(src + (size_t)l * g.ps + g.origin + (long long)xs * g.cs - EY[l], yb);
    }
    if constexpr (sizeof(S) == 8) {
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
    }
    S* col = dst + g.origin + (long long)x * g.cs;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_nt(col + (size_t)l * g.ps, yb, f[l]);
}

template <typename L, int T = lbm::adj_threads<L>()>
__global__ __launch_bounds__(T) void k_adjoint_pattern(const float* __restrict__ f, const L* __restrict__ lam,
                                                       L* __restrict__ mu, lbm::Geo g, lbm::Geo lg)
{
    using namespace lbm;
    const SiteBlock sb = site_block<true, T>(g);
    const int x = sb.x, y = sb.y;
    if (y >= g.ly) return;
    const unsigned yb = (unsigned)y * 4u, yd = (unsigned)y * (unsigned)sizeof(L);
    float gl[NPOP];
    L la[NPOP];
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        la[l] = ld_at(lam + (size_t)l * lg.ps + lg.origin + (long long)wrap_x(x + EX[l], lg.lx) * lg.cs + EY[l], yd);
    }
#pragma unroll
    for (int l = 0; l < NPOP; ++l) {
        gl[l] = ld_at(f + (size_t)l * g.ps + g.origin + (long long)wrap_x(x - EX[l], g.lx) * g.cs - EY[l], yb);
    }
    L* mcol = mu + lg.origin + (long long)x * lg.cs;
#pragma unroll
    for (int l = 0; l < NPOP; ++l) st_nt(mcol + (size_t)l * lg.ps, yd, (L)(la[l] + (L)gl[l]));
}

bool gather_args_ok(int elem_bytes, int lx, int ly)
{
    return (elem_bytes == 8 || elem_bytes == 4) && lx >= 7 && ly >= 7 && (long long)lx * ly <= (1LL << 31);
}

typedef double v2 __attribute__((ext_vector_type(2)));

template <int T>
__global__ __launch_bounds__(T) void k_copy(const v2* __restrict__ src, v2* __restrict__ dst, size_t n)
{
    const size_t b = (size_t)blockIdx.x * T;
    if (b + threadIdx.x < n)
        lbm::st_nt<v2>(dst + b, threadIdx.x * 16u, __builtin_nontemporal_load(src + b + threadIdx.x));
}

template <int T>
int launch(const void* src, void* dst, size_t n, hipStream_t s)
{
    const size_t nb = (n + T - 1) / T;
    if (nb * T > 0xffffffffull) return 1;   // grid size in work-items must fit 32 bits
    hipLaunchKernelGGL((k_copy<T>), dim3((unsigned)nb), dim3(T), 0, s, (const v2*)src, (v2*)dst, n);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // namespace

extern "C" int cp_copy(const void* src, void* dst, size_t bytes, int block_bytes, void* stream)
{
    if (!src || !dst || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return 1;
    const char* a = (const char*)src;
    const char* b = (const char*)dst;
    if (a < b + bytes && b < a + bytes) return 1;   // overlapping ranges
    const size_t n = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
    switch (block_bytes) {
    case 1024: return launch<64>(src, dst, n, s);
    case 2048: return launch<128>(src, dst, n, s);
    case 4096: return launch<256>(src, dst, n, s);
    default: return 1;
    }
}

extern "C" size_t cp_gather_bytes(int elem_bytes, int lx, int ly)
{
    if (!gather_args_ok(elem_bytes, lx, ly)) return 0;
    return (size_t)lbm::padded_geo(lx, ly, (size_t)elem_bytes, false).total * (size_t)elem_bytes;
}

extern "C" int cp_gather_copy(int elem_bytes, int lx, int ly, const void* src, void* dst, void* stream)
{
    if (!gather_args_ok(elem_bytes, lx, ly) || !src || !dst || src == dst ||
        ((uintptr_t)src | (uintptr_t)dst) % 256 != 0)
        return 1;
    const lbm::Geo g = lbm::padded_geo(lx, ly, (size_t)elem_bytes, false);
    const size_t bytes = (size_t)g.total * (size_t)elem_bytes;
    const char* a = (const char*)src;
    const char* b = (const char*)dst;
    if (a < b + bytes && b < a + bytes) return 1;   // overlapping buffers
    const dim3 grid((unsigned)((ly + lbm::SITE_THREADS - 1) / lbm::SITE_THREADS) * (unsigned)lx);
    hipStream_t s = (hipStream_t)stream;
    if (elem_bytes == 4) {
        hipLaunchKernelGGL((k_gather_copy<float>), grid, dim3(lbm::SITE_THREADS), 0, s, (const float*)src,
                           (float*)dst, g);
        return hipGetLastError() == hipSuccess ? 0 : 2;
    }
    // the FP64 fused step's launch settings (lbm_kernels.hpp), by the same rule
    lbm::FusedLaunch fl{lbm::SITE_THREADS, 0u};
    int dev = 0, ncu = 0, max_lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
        fl = lbm::fused_fp64_launch(grid.x, ncu, max_lds);
    if (fl.threads == lbm::FUSED_FP64_WIDE_THREADS) {
        constexpr int T = lbm::FUSED_FP64_WIDE_THREADS;
        const dim3 wgrid((unsigned)((ly + T - 1) / T) * (unsigned)lx);
        hipLaunchKernelGGL((k_gather_copy<double, T>), wgrid, dim3(T), fl.lds, s, (const double*)src,
                           (double*)dst, g);
    } else {
        hipLaunchKernelGGL((k_gather_copy<double>), grid, dim3(lbm::SITE_THREADS), fl.lds, s, (const double*)src,
                           (double*)dst, g);
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int cp_adjoint_pattern(int lam_bytes, int lx, int ly, const void* f, const void* lam, void* mu,
                                  void* stream)
{
    if (!gather_args_ok(lam_bytes, lx, ly) || !f || !lam || !mu || f == lam || f == mu || lam == mu ||
        ((uintptr_t)f | (uintptr_t)lam | (uintptr_t)mu) % 256 != 0)
        return 1;
    const lbm::Geo g = lbm::padded_geo(lx, ly, 4, false);
    const lbm::Geo lg = lbm::padded_geo(lx, ly, (size_t)lam_bytes, false);
    const size_t nf = (size_t)g.total * 4, nl = (size_t)lg.total * (size_t)lam_bytes;
    auto overlap = [](const void* p, size_t n, const void* q, size_t m) {
        const char* a = (const char*)p;
        const char* b = (const char*)q;
        return a < b + m && b < a + n;
    };
    if (overlap(f, nf, lam, nl) || overlap(f, nf, mu, nl) || overlap(lam, nl, mu, nl)) return 1;
    hipStream_t s = (hipStream_t)stream;
    // the reverse step's block size for this lambda storage
    if (lam_bytes == 8) {
        constexpr int T = lbm::adj_threads<double>();
        const dim3 grid((unsigned)((ly + T - 1) / T) * (unsigned)lx);
        hipLaunchKernelGGL((k_adjoint_pattern<double>), grid, dim3(T), 0, s, (const float*)f, (const double*)lam,
                           (double*)mu, g, lg);
    } else {
        constexpr int T = lbm::adj_threads<float>();
        const dim3 grid((unsigned)((ly + T - 1) / T) * (unsigned)lx);
        hipLaunchKernelGGL((k_adjoint_pattern<float>), grid, dim3(T), 0, s, (const float*)f, (const float*)lam,
                           (float*)mu, g, lg);
    }
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
