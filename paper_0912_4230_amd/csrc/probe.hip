// probe.hip -- measurement kernels, built into their own library
// (libporolbm_probe.so) and run only by profile_run: not part of the lattice
// library or its C ABI.
//
// probe_copy_f4: a streaming copy of float4 elements with the non-temporal
// load and store policy of the step kernel's population streams, one grid
// that strides over the buffer.  Its rate is the practical HBM ceiling of a
// read-once / write-once stream on this part, which the step's achieved
// bandwidth is compared with.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy_f4(f4 *__restrict__ dst, const f4 *__restrict__ src, size_t n)
{
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const f4 v = __builtin_nontemporal_load(src + i);
        __builtin_nontemporal_store(v, dst + i);
    }
}

// NS streams per thread, the access pattern of a step's population planes
// without the stencil shifts: thread i reads element i of each of the NS
// source planes (all loads issued first) and writes it to the same place in
// the destination copy.  Plane-major layout (slice == 0): element i of plane k
// at k * pstride + i.  Slice-major layout: the cells are cut into slices of
// `slice` cells (one z-plane of the lattice) and element i of plane k is at
// ((i / slice) * NS + k) * sstride + i % slice, i.e. all NS planes of a slice
// are contiguous.
template <int NS, class T>
__global__ __launch_bounds__(256) void k_streams(T *__restrict__ dst, const T *__restrict__ src, size_t n,
                                                 size_t pstride, size_t slice, size_t sstride)
{
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t base, step;
    if (slice == 0) {
        base = i;
        step = pstride;
    } else {
        base = (i / slice) * NS * sstride + i % slice;
        step = sstride;
    }
    T v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = __builtin_nontemporal_load(src + base + k * step);
#pragma unroll
    for (int k = 0; k < NS; ++k) __builtin_nontemporal_store(v[k], dst + base + k * step);
}

}  // namespace

extern "C" {

// k_streams<38> over n cells (one cell per thread) of elements of `elem`
// bytes (4 or 2): src and dst each hold 38 planes in the given layout (the
// caller sizes them: plane-major 38 * pstride elements, slice-major
// ceil(n / slice) * 38 * sstride elements).  Returns 0, or 1 on a rejected
// argument, 2 on a launch error.  Asynchronous.
int probe_streams38(void *dst, const void *src, size_t n, size_t pstride, size_t slice, size_t sstride,
                    void *stream, int elem)
{
    if (!dst || !src || n == 0 || (elem != 4 && elem != 2)) return 1;
    if (slice == 0 ? pstride < n : sstride < slice) return 1;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (elem == 4)
        hipLaunchKernelGGL((k_streams<38, float>), dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<float *>(dst),
                           static_cast<const float *>(src), n, pstride, slice, sstride);
    else
        hipLaunchKernelGGL((k_streams<38, uint16_t>), dim3(unsigned(blocks)), dim3(256), 0, s,
                           static_cast<uint16_t *>(dst), static_cast<const uint16_t *>(src), n, pstride, slice, sstride);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

// Copy `bytes` (a multiple of 16; both pointers 16-byte aligned device
// pointers) with `blocks` blocks of 256 threads on `stream` (a hipStream_t,
// NULL: default).  Returns 0, or 1 on a rejected argument, 2 on a launch
// error.  Asynchronous.
int probe_copy_f4(void *dst, const void *src, size_t bytes, void *stream, int blocks)
{
    if (!dst || !src || bytes % 16 || blocks <= 0) return 1;
    if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16) return 1;
    hipLaunchKernelGGL(k_copy_f4, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<f4 *>(dst), static_cast<const f4 *>(src), bytes / 16);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
