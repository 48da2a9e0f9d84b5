// Self-check of the projection's reciprocal (declared in include/rz.h):
// the kernels compute the perspective divide's 1 / w (section 2.1, in
// single precision) as a Newton-corrected hardware estimate with a
// fallback to the IEEE division; this compares that function, as compiled
// into the library, with the IEEE quotient over a range of float bit
// patterns on the current device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_device.h"
#include "rz_internal.h"

namespace rz {

int hip_fail(hipError_t e);

namespace {

constexpr int kCheckBlock = 256;
constexpr int64_t kCheckMaxBlocks = 65536;

template <bool FULL>
__global__ void __launch_bounds__(kCheckBlock) k_check_recip(uint32_t first, int64_t count,
                                                             unsigned long long *mismatches)
{
    const int64_t stride = (int64_t)gridDim.x * kCheckBlock;
    unsigned long long bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kCheckBlock + threadIdx.x; i < count; i += stride) {
        const float w = __uint_as_float(first + (uint32_t)i);
        const float got = FULL ? dev::recip_rn(w) : dev::recip_newton(w);
        const float want = 1.0f / w;
        bad += (w > 0.0f) & (__float_as_uint(got) != __float_as_uint(want));
    }
    if (bad)
        atomicAdd(mismatches, bad);
}

// The same device function over caller-given values, results to memory, so
// that a host can compare them with its own IEEE quotients.
__global__ void __launch_bounds__(kCheckBlock) k_recip_values(const float *__restrict__ w,
                                                              float *__restrict__ out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kCheckBlock;
    for (int64_t i = (int64_t)blockIdx.x * kCheckBlock + threadIdx.x; i < n; i += stride)
        out[i] = dev::recip_rn(w[i]);
}

}  // namespace
}  // namespace rz

using namespace rz;

extern "C" int rz_check_reciprocal(uint32_t first_bits, int64_t count, uint64_t *mismatches,
                                   uint32_t flags, void *stream)
{
    if ((flags & ~RZ_CHECK_ESTIMATE_ONLY) || count < 0 ||
        (uint64_t)first_bits + (uint64_t)count > (1ull << 32) || !mismatches ||
        ((uintptr_t)mismatches & 7u))
        return RZ_EINVAL;
    if (count == 0)
        return RZ_OK;
    int64_t blocks = (count + kCheckBlock - 1) / kCheckBlock;
    blocks = blocks < kCheckMaxBlocks ? blocks : kCheckMaxBlocks;
    unsigned long long *out = reinterpret_cast<unsigned long long *>(mismatches);
    if (flags & RZ_CHECK_ESTIMATE_ONLY)
        hipLaunchKernelGGL(k_check_recip<false>, dim3((uint32_t)blocks), dim3(kCheckBlock), 0,
                           (hipStream_t)stream, first_bits, count, out);
    else
        hipLaunchKernelGGL(k_check_recip<true>, dim3((uint32_t)blocks), dim3(kCheckBlock), 0,
                           (hipStream_t)stream, first_bits, count, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

extern "C" int rz_reciprocal(const float *w, float *out, int64_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!w || !out)))
        return RZ_EINVAL;
    if (n == 0)
        return RZ_OK;
    int64_t blocks = (n + kCheckBlock - 1) / kCheckBlock;
    blocks = blocks < kCheckMaxBlocks ? blocks : kCheckMaxBlocks;
    hipLaunchKernelGGL(k_recip_values, dim3((uint32_t)blocks), dim3(kCheckBlock), 0,
                       (hipStream_t)stream, w, out, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}
