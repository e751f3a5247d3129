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


// The D3Q19 link vectors in the order of the lattice library (rest, the six
// axis links, the twelve diagonal links); only the shifts matter here.
__constant__ int c_probe_v[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                                     {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                                     {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

// 38 streams over a periodic cube of (1 << lg)^3 cells, one cell per thread:
// stream k reads the value of cell x - v_(k mod 19) (SHIFT, the pull of a
// lattice step; else x itself) and writes cell x.  Plane-major layout (ROW =
// false): element of cell j in stream k at k * pstride + j.  Row-interleaved
// layout (ROW = true): every row of cells (fixed y and z) holds its 38 streams
// one after the other, each `pitch` elements long: cell (x, y, z) of stream k
// at (row * 38 + k) * pitch + x with row = y + z * 2^lg.  XG: block b of the
// grid (XCD b mod 8) takes logical block (s / 4) * 32 + (b mod 8) * 4 + s mod 4,
// s = b / 8, so that each XCD sweeps runs of 4 consecutive blocks (the row
// groups of the lattice step; the grid is a multiple of 32 blocks).
template <class T, bool ROW, bool SHIFT, bool XG>
__global__ __launch_bounds__(256) void k_streams_shift(T *__restrict__ dst, const T *__restrict__ src, int lg,
                                                       size_t pstride, size_t pitch)
{
    size_t blk = blockIdx.x;
    if constexpr (XG) blk = ((blk >> 3) / 4) * 32 + (blk & 7) * 4 + ((blk >> 3) % 4);
    const size_t i = blk * blockDim.x + threadIdx.x;
    const size_t m = (size_t(1) << lg) - 1;
    if (i > (m << (2 * lg)) + (m << lg) + m) return;
    const size_t x = i & m, y = (i >> lg) & m, z = i >> (2 * lg);
    T v[38];
#pragma unroll
    for (int k = 0; k < 38; ++k) {
        size_t xs = x, ys = y, zs = z;
        if constexpr (SHIFT) {
            xs = (x - size_t(c_probe_v[k % 19][0])) & m;
            ys = (y - size_t(c_probe_v[k % 19][1])) & m;
            zs = (z - size_t(c_probe_v[k % 19][2])) & m;
        }
        const size_t at = ROW ? (((zs << lg) + ys) * 38 + k) * pitch + xs : k * pstride + (((zs << lg) + ys) << lg) + xs;
        v[k] = __builtin_nontemporal_load(src + at);
    }
#pragma unroll
    for (int k = 0; k < 38; ++k) {
        const size_t at = ROW ? (((z << lg) + y) * 38 + k) * pitch + x : k * pstride + i;
        __builtin_nontemporal_store(v[k], dst + at);
    }
}

// NS streams (38, or 19 of elements twice as wide: the two lattices' values
// of a link side by side) with the pull of k_streams_shift and its XCD row
// groups, addressed as the lattice step addresses its planes: a block is 256
// cells of one row (2^lg >= 256), so y and z are uniform over it and every
// stream's source row is one uniform base; a lane adds only its 32-bit x
// offset.  The z neighbours are clamped at the cube's faces instead of wrapped
// (only the access pattern matters).  ROW: the row-interleaved layout of
// k_streams_shift (NS streams per row).
template <class T, bool ROW, int NS>
__global__ __launch_bounds__(256) void k_streams_uni(T *__restrict__ dst, const T *__restrict__ src, int lg,
                                                     size_t pstride, size_t pitch)
{
    int blk = blockIdx.x;
    blk = ((blk >> 3) / 4) * 32 + (blk & 7) * 4 + ((blk >> 3) % 4);
    const int m = (1 << lg) - 1;
    const int bpr = 1 << (lg - 8);                       // blocks per row
    const int row = blk / bpr;                           // uniform
    const int y = row & m, z = row >> lg;
    const uint32_t x = uint32_t((blk % bpr) * 256 + threadIdx.x);
    T v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int ys = (y - c_probe_v[k % 19][1]) & m;
        const int zs = min(max(z - c_probe_v[k % 19][2], 0), m);
        const uint32_t xs = (x - uint32_t(c_probe_v[k % 19][0])) & uint32_t(m);
        const size_t srow = (size_t(zs) << lg) + size_t(ys);
        const T *base = ROW ? src + (srow * NS + k) * pitch : src + k * pstride + (srow << lg);
        v[k] = __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                                                      xs * uint32_t(sizeof(T))));
    }
    const size_t orow = (size_t(z) << lg) + size_t(y);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T *base = ROW ? dst + (orow * NS + k) * pitch : dst + k * pstride + (orow << lg);
        __builtin_nontemporal_store(v[k], reinterpret_cast<T *>(reinterpret_cast<char *>(base) + x * uint32_t(sizeof(T))));
    }
}

template <class T, int NS>
int launch_uni(void *dst, const void *src, int lg, int row, size_t pstride, size_t pitch, hipStream_t s)
{
    const size_t nb = (size_t(1) << (3 * lg)) / 256;
    T *d = static_cast<T *>(dst);
    const T *r = static_cast<const T *>(src);
    if (row) hipLaunchKernelGGL((k_streams_uni<T, true, NS>), dim3(unsigned(nb)), dim3(256), 0, s, d, r, lg, pstride, pitch);
    else hipLaunchKernelGGL((k_streams_uni<T, false, NS>), dim3(unsigned(nb)), dim3(256), 0, s, d, r, lg, pstride, pitch);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

// NS streams of one copy read and written in place (the two kinds of step
// of an in-place streaming scheme), with the XCD row groups and uniform row
// bases of k_streams_uni, over a periodic cube of 2^lg cells per edge
// (2^lg >= 256).  ODD: stream k of cell x reads and writes the element of
// cell x - v_(k mod 19) (every element is touched by exactly one thread: the
// shift is a bijection of the periodic cube); else the element of cell x
// itself.  The value written is the value read plus one.
template <class T, int NS, bool ODD>
__global__ __launch_bounds__(256) void k_streams_aa(T *__restrict__ buf, int lg, size_t pstride)
{
    int blk = blockIdx.x;
    blk = ((blk >> 3) / 4) * 32 + (blk & 7) * 4 + ((blk >> 3) % 4);
    const int m = (1 << lg) - 1;
    const int bpr = 1 << (lg - 8);
    const int row = blk / bpr;
    const int y = row & m, z = row >> lg;
    const uint32_t x = uint32_t((blk % bpr) * 256 + threadIdx.x);
    T v[NS];
    uint32_t off[NS];
    T *base[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        int ys = y, zs = z;
        uint32_t xs = x;
        if constexpr (ODD) {
            ys = (y - c_probe_v[k % 19][1]) & m;
            zs = (z - c_probe_v[k % 19][2]) & m;
            xs = (x - uint32_t(c_probe_v[k % 19][0])) & uint32_t(m);
        }
        base[k] = buf + k * pstride + (((size_t(zs) << lg) + size_t(ys)) << lg);
        off[k] = xs * uint32_t(sizeof(T));
        v[k] = __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base[k]) + off[k]));
    }
#pragma unroll
    for (int k = 0; k < NS; ++k)
        __builtin_nontemporal_store(T(v[k] + T(1)), reinterpret_cast<T *>(reinterpret_cast<char *>(base[k]) + off[k]));
}

template <class T, bool XG>
void launch_shift_xg(T *d, const T *r, int lg, int row, int shift, size_t pstride, size_t pitch, dim3 grid,
                     hipStream_t s)
{
    const dim3 block(256);
    if (row && shift) hipLaunchKernelGGL((k_streams_shift<T, true, true, XG>), grid, block, 0, s, d, r, lg, pstride, pitch);
    else if (row) hipLaunchKernelGGL((k_streams_shift<T, true, false, XG>), grid, block, 0, s, d, r, lg, pstride, pitch);
    else if (shift) hipLaunchKernelGGL((k_streams_shift<T, false, true, XG>), grid, block, 0, s, d, r, lg, pstride, pitch);
    else hipLaunchKernelGGL((k_streams_shift<T, false, false, XG>), grid, block, 0, s, d, r, lg, pstride, pitch);
}

template <class T>
int launch_shift(void *dst, const void *src, int lg, int row, int shift, int xg, size_t pstride, size_t pitch,
                 hipStream_t s)
{
    const size_t n = size_t(1) << (3 * lg);
    const size_t nb = (n + 255) / 256;
    if (xg && nb % 32 != 0) return 1;
    T *d = static_cast<T *>(dst);
    const T *r = static_cast<const T *>(src);
    if (xg == 2) {
        if (lg < 8) return 1;
        return launch_uni<T, 38>(dst, src, lg, row, pstride, pitch, s);
    } else if (xg) launch_shift_xg<T, true>(d, r, lg, row, shift, pstride, pitch, dim3(unsigned(nb)), s);
    else launch_shift_xg<T, false>(d, r, lg, row, shift, pstride, pitch, dim3(unsigned(nb)), s);
    return hipGetLastError() == hipSuccess ? 0 : 2;
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

// k_streams_shift over a periodic cube of 2^lg cells per edge (2 <= lg <= 9)
// of `elem`-byte elements (4 or 2): row = 0 plane-major (the caller sizes src
// and dst to 38 * pstride elements, pstride >= 2^(3 lg)), row = 1
// row-interleaved (38 * 2^(2 lg) * pitch elements, pitch >= 2^lg); shift = 1
// pulls every stream from the upstream cell of its link; xg = 1 maps the
// blocks to XCD row groups (2^(3 lg) a multiple of 8192); xg = 2 runs
// k_streams_uni (shifted, XCD row groups, uniform row bases; lg >= 8).  Returns 0, or 1 on
// a rejected argument, 2 on a launch error.  Asynchronous.
int probe_streams38_cube(void *dst, const void *src, int lg, int row, int shift, int xg, size_t pstride,
                         size_t pitch, void *stream, int elem)
{
    if (!dst || !src || lg < 2 || lg > 9 || (elem != 4 && elem != 2)) return 1;
    const size_t n = size_t(1) << (3 * lg);
    if (row ? pitch < (size_t(1) << lg) : pstride < n) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return elem == 4 ? launch_shift<float>(dst, src, lg, row, shift, xg, pstride, pitch, s)
                     : launch_shift<uint16_t>(dst, src, lg, row, shift, xg, pstride, pitch, s);
}

// k_streams_uni with ns = 19 streams of elem = 4 or 8 bytes (the two
// lattices' 2- or 4-byte values of a link side by side) or ns = 38 of 2 or 4
// bytes, over a cube of 2^lg cells per edge (8 <= lg <= 9): row = 0
// plane-major (src and dst ns * pstride elements, pstride >= 2^(3 lg)), row = 1
// row-interleaved (ns * 2^(2 lg) * pitch elements, pitch >= 2^lg).  Returns 0,
// or 1 on a rejected argument, 2 on a launch error.  Asynchronous.
int probe_streams_uni(void *dst, const void *src, int lg, int ns, int row, size_t pstride, size_t pitch,
                      void *stream, int elem)
{
    if (!dst || !src || lg < 8 || lg > 9) return 1;
    const size_t n = size_t(1) << (3 * lg);
    if (row ? pitch < (size_t(1) << lg) : pstride < n) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ns == 19 && elem == 8) return launch_uni<uint64_t, 19>(dst, src, lg, row, pstride, pitch, s);
    if (ns == 19 && elem == 4) return launch_uni<uint32_t, 19>(dst, src, lg, row, pstride, pitch, s);
    if (ns == 38 && elem == 4) return launch_uni<uint32_t, 38>(dst, src, lg, row, pstride, pitch, s);
    if (ns == 38 && elem == 2) return launch_uni<uint16_t, 38>(dst, src, lg, row, pstride, pitch, s);
    return 1;
}

// k_streams_aa: ns = 38 or 19 streams of 4-byte elements read and written in
// place in one plane-major copy (ns * pstride elements, pstride >= 2^(3 lg)),
// odd = 1 shifted, 0 local, over a cube of 2^lg cells per edge (8 <= lg <= 9).
// Returns 0, or 1 on a rejected argument, 2 on a launch error.  Asynchronous.
int probe_streams_aa(void *buf, int lg, int ns, int odd, size_t pstride, void *stream)
{
    if (!buf || lg < 8 || lg > 9 || (ns != 38 && ns != 19)) return 1;
    const size_t n = size_t(1) << (3 * lg);
    if (pstride < n) return 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid(unsigned(n / 256)), block(256);
    uint32_t *b = static_cast<uint32_t *>(buf);
    if (ns == 38 && odd) hipLaunchKernelGGL((k_streams_aa<uint32_t, 38, true>), grid, block, 0, s, b, lg, pstride);
    else if (ns == 38) hipLaunchKernelGGL((k_streams_aa<uint32_t, 38, false>), grid, block, 0, s, b, lg, pstride);
    else if (odd) hipLaunchKernelGGL((k_streams_aa<uint32_t, 19, true>), grid, block, 0, s, b, lg, pstride);
    else hipLaunchKernelGGL((k_streams_aa<uint32_t, 19, false>), grid, block, 0, s, b, lg, pstride);
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
