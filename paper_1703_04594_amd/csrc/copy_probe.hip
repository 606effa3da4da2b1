// copy_probe.hip -- reference streaming copy for roofline calibration.
//
// Not part of the lattice Boltzmann path: the benchmark times it beside
// propagate, on a buffer the size of one population buffer, so that
// propagate's bandwidth can be quoted as a fraction of a plain copy measured
// on the same GPU in the same run.  dst[i] = src[i] over `bytes` bytes in
// 16-byte vectors, one workgroup per chunk of `block_bytes` bytes (1024, 2048
// or 4096: 64, 128 or 256 threads), non-temporal loads and stores, hardware
// block order (the fastest plain copy measured on MI355X used this form).
//
// int cp_copy(const void* src, void* dst, size_t bytes, int block_bytes,
//             void* hip_stream)
//   src, dst: device pointers, 16-byte aligned, not overlapping; bytes a
//   multiple of 16.  Enqueued on hip_stream (a hipStream_t, 0 = default
//   stream); returns without waiting.  Returns 0 on success, 1 for an invalid
//   argument (nothing launched), 2 if the launch failed.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

typedef double v2 __attribute__((ext_vector_type(2)));

template <int T>
__global__ __launch_bounds__(T) void k_copy(const v2* __restrict__ src, v2* __restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * T + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
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
