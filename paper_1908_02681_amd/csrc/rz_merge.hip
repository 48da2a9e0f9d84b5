// Sort-last composition (declared in include/rz.h): per-pixel minimum of
// two framebuffers (section 2.1) and sum of two packed splat accumulators
// (section 2.2).  Streaming kernels: two pixels of keys, or one pixel of
// sums, per 16-byte load; the HBM bound is 24 B/pixel for the minimum and
// 48 B/pixel for the sums.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rz.h"
#include "rz_internal.h"
#include "rz_trace.h"

namespace rz {

int hip_fail(hipError_t e);

namespace {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

constexpr int kMergeBlock = 256;

__global__ void __launch_bounds__(kMergeBlock) k_merge_min(uint64_t *__restrict__ dst,
                                                           const uint64_t *__restrict__ src,
                                                           int64_t npix)
{
    const int64_t i = 2 * ((int64_t)blockIdx.x * kMergeBlock + threadIdx.x);
    if (i + 1 < npix) {
        u64x2 a = *reinterpret_cast<const u64x2 *>(dst + i);
        const u64x2 b = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(src + i));
        a.x = b.x < a.x ? b.x : a.x;
        a.y = b.y < a.y ? b.y : a.y;
        *reinterpret_cast<u64x2 *>(dst + i) = a;
    } else if (i < npix) {
        dst[i] = src[i] < dst[i] ? src[i] : dst[i];
    }
}

__global__ void __launch_bounds__(kMergeBlock) k_merge_sum(uint64_t *__restrict__ dst,
                                                           const uint64_t *__restrict__ src,
                                                           int64_t npix)
{
    const int64_t p = (int64_t)blockIdx.x * kMergeBlock + threadIdx.x;
    if (p >= npix)
        return;
    u64x2 a = *reinterpret_cast<const u64x2 *>(dst + 2 * p);
    const u64x2 b = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(src + 2 * p));
    a += b;
    *reinterpret_cast<u64x2 *>(dst + 2 * p) = a;
}

bool aligned(const void *a, size_t n) { return ((uintptr_t)a & (n - 1)) == 0; }

// [a, a + na) and [b, b + nb) (bytes) overlap
bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace
}  // namespace rz

using namespace rz;

extern "C" {

int rz_merge_min(uint64_t *dst, const uint64_t *src, int64_t npix, void *stream)
{
    Range range("rz_merge_min");
    if (npix < 0)
        return RZ_EINVAL;
    if (npix == 0)
        return RZ_OK;
    if (!dst || !src || !aligned(dst, 16) || !aligned(src, 16) ||
        overlap(dst, (size_t)npix * 8, src, (size_t)npix * 8))
        return RZ_EINVAL;
    const int64_t threads = (npix + 1) / 2;
    hipLaunchKernelGGL(k_merge_min, dim3((uint32_t)((threads + kMergeBlock - 1) / kMergeBlock)),
                       dim3(kMergeBlock), 0, (hipStream_t)stream, dst, src, npix);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

int rz_merge_sum(uint64_t *dst, const uint64_t *src, int64_t npix, void *stream)
{
    Range range("rz_merge_sum");
    if (npix < 0)
        return RZ_EINVAL;
    if (npix == 0)
        return RZ_OK;
    if (!dst || !src || !aligned(dst, 16) || !aligned(src, 16) ||
        overlap(dst, (size_t)npix * 16, src, (size_t)npix * 16))
        return RZ_EINVAL;
    hipLaunchKernelGGL(k_merge_sum, dim3((uint32_t)((npix + kMergeBlock - 1) / kMergeBlock)),
                       dim3(kMergeBlock), 0, (hipStream_t)stream, dst, src, npix);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RZ_OK : hip_fail(e);
}

}  // extern "C"
