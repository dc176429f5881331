// pdn_copy.hip -- streaming device copy: the HBM bandwidth ceiling that the
// element/node kernel's roofline fraction is read against (a measurement
// hook, not a step of the method).
//
// Each lane moves four 16-byte words per iteration, the four loads issued
// before the stores, with consecutive lanes on consecutive words (every wave
// access is one contiguous 1 KiB run); the grid strides over the buffer.
#include "pdn.h"

#include <hip/hip_runtime.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                     int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(src + i);
        const u32x4 b = __builtin_nontemporal_load(src + i + stride);
        const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" int pdn_stream_copy(int32_t device, void *stream, const void *src, void *dst, int64_t bytes)
{
    if (!src || !dst || bytes < 0 || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return PDN_EINVAL;
    if (bytes == 0) return PDN_OK;
    if (hipSetDevice(device) != hipSuccess) return PDN_EDEVICE;
    const int64_t n16 = bytes / 16;
    // 256 CUs x 8 workgroups of 256 lanes, or fewer for small buffers
    int64_t blocks = (n16 + 4 * 256 - 1) / (4 * 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const u32x4 *)src, (u32x4 *)dst, n16);
    return hipGetLastError() == hipSuccess ? PDN_OK : PDN_EDEVICE;
}
