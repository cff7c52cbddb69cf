// reduce.hip -- per-pattern compensated complex FP64 reduction.
//
// One 256-thread block per pattern.  Each thread keeps a TwoSum-compensated
// running sum (value, error) of a strided share of the pattern's entries; the
// 64 lanes of a wave then combine their pairs with a fixed butterfly of
// cross-lane shuffles (error terms carried along), the four waves combine in
// LDS in a fixed order, and the final value is sum + error.  The order of
// every addition depends only on the entry count, so the result is
// bit-reproducible and independent of what else runs on the GPU.
#include "lofp_device.h"

namespace lofp {

__device__ __forceinline__ CSum wave_combine(CSum a)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        CSum b;
        b.s = __shfl_xor(a.s, off, 64);
        b.c = __shfl_xor(a.c, off, 64);
        // both partners must add in the same order to stay bit-identical
        const int lane = threadIdx.x & 63;
        if (lane & off) { CSum t = a; a = b; b = t; }
        csum_merge(a, b);
    }
    return a;
}

template <bool DOT>
__global__ __launch_bounds__(256) void k_reduce(int B, const int64_t *__restrict__ off,
                                                const double2 *__restrict__ vec,
                                                const double2 *__restrict__ back, double2 *__restrict__ out)
{
    const int p = blockIdx.x;
    const int64_t beg = off[p], end = off[p + 1];
    CSum sr{0.0, 0.0}, si{0.0, 0.0};
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        double2 x = vec[i];
        if (DOT) x = cmul(x, back[i]);
        csum_add(sr, x.x);
        csum_add(si, x.y);
    }
    sr = wave_combine(sr);
    si = wave_combine(si);
    __shared__ CSum part[2][4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { part[0][wv] = sr; part[1][wv] = si; }
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum r = part[0][0], q = part[1][0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) { csum_merge(r, part[0][w]); csum_merge(q, part[1][w]); }
        out[p] = make_double2(r.s + r.c, q.s + q.c);
    }
}

hipError_t launch_reduce(int B, const int64_t *off, const double2 *vec, const double2 *back, double2 *out,
                         hipStream_t stream)
{
    if (B == 0) return hipSuccess;
    if (back) hipLaunchKernelGGL((k_reduce<true>), dim3(B), dim3(256), 0, stream, B, off, vec, back, out);
    else hipLaunchKernelGGL((k_reduce<false>), dim3(B), dim3(256), 0, stream, B, off, vec, back, out);
    return hipGetLastError();
}

}  // namespace lofp
