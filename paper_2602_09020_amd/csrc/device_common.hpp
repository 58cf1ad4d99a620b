// Device helpers shared by the single-state kernels and the batched kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfh {
namespace dev {

// Amplitudes are stored as double2 (complex128) or float2 (complex64) and
// always processed as double2 in registers.
__device__ __forceinline__ double2 ld(const double2 &p) { return p; }
__device__ __forceinline__ double2 ld(const float2 &p) { return make_double2(p.x, p.y); }
__device__ __forceinline__ void st(double2 &p, double2 v) { p = v; }
__device__ __forceinline__ void st(float2 &p, double2 v) { p = make_float2((float)v.x, (float)v.y); }

__device__ __forceinline__ int par32(uint32_t v) { return __builtin_popcount(v) & 1; }
__device__ __forceinline__ int par64(uint64_t v) { return __builtin_popcountll(v) & 1; }

// Spread the low bits of v over the set bits of mask (software pdep).
__device__ __forceinline__ uint64_t deposit(uint64_t v, uint64_t mask)
{
    uint64_t r = 0;
    for (uint64_t m = mask; m && v; m &= m - 1, v >>= 1)
        if (v & 1) r |= m & (~m + 1);
    return r;
}

// One pair update of exp(-i theta/2 P): with beta = sr * (imag ? i : 1),
//   u' = c u + s0 beta v,  v' = c v + s1 beta u,  the member signs folded into s0, s1.
__device__ __forceinline__ void rot_pair(double2 &u, double2 &v, double c, double s0, double s1, bool imag)
{
    double2 nu, nv;
    if (imag) {
        nu.x = c * u.x - s0 * v.y;
        nu.y = c * u.y + s0 * v.x;
        nv.x = c * v.x - s1 * u.y;
        nv.y = c * v.y + s1 * u.x;
    } else {
        nu.x = c * u.x + s0 * v.x;
        nu.y = c * u.y + s0 * v.y;
        nv.x = c * v.x + s1 * u.x;
        nv.y = c * v.y + s1 * u.y;
    }
    u = nu;
    v = nv;
}

// Diagonal member update: u' = (c + s beta) u.
__device__ __forceinline__ double2 rot_diag(double2 u, double c, double s, bool imag)
{
    if (imag) return make_double2(c * u.x - s * u.y, c * u.y + s * u.x);
    return make_double2((c + s) * u.x, (c + s) * u.y);
}

// Sum over the first WIDTH lanes of a wave (WIDTH = min(block size, 64)).
template <int WIDTH>
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = WIDTH / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WIDTH);
    return v;
}

} // namespace dev
} // namespace cfh
