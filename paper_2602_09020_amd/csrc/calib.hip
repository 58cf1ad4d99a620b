// Calibration kernels: the HBM rate that an in-place update of a
// state-sized buffer reaches on this device.  Every amplitude is read once,
// multiplied by a fixed unit phase and written back, one amplitude per thread
// and one short-lived workgroup per 256 amplitudes, so the hardware
// dispatcher keeps the whole chip streaming.  The scattered form permutes
// the index bits above the chunk (bit-reversed), so runs of 2^chunk_bits
// contiguous amplitudes land far apart, which is the access pattern of a
// fused pass over GF(2) coset tiles whose free dimensions are high qubits.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cfh_internal.hpp"
#include "launch.hpp"

using namespace cfh;

namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double2 ld_amp(const double2 *p, bool nt)
{
    if (nt) {
        const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(p));
        return make_double2(v.x, v.y);
    }
    return *p;
}
__device__ __forceinline__ double2 ld_amp(const float2 *p, bool nt)
{
    if (nt) {
        const fvec2 v = __builtin_nontemporal_load(reinterpret_cast<const fvec2 *>(p));
        return make_double2(v.x, v.y);
    }
    return make_double2(p->x, p->y);
}
__device__ __forceinline__ void st_amp(double2 *p, double2 v, bool nt)
{
    if (nt) {
        const dvec2 w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<dvec2 *>(p));
    } else {
        *p = v;
    }
}
__device__ __forceinline__ void st_amp(float2 *p, double2 v, bool nt)
{
    if (nt) {
        const fvec2 w = {(float)v.x, (float)v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<fvec2 *>(p));
    } else {
        *p = make_float2((float)v.x, (float)v.y);
    }
}

// Thread i updates amplitude a(i): a = i (contiguous), or with the index
// bits above the low cbits bit-reversed (scattered chunks).  The launches
// together cover i in [0, 2^nbits) exactly once (i0 is a launch's first i), so
// a(i) is a permutation of [0, 2^nbits).
template <typename Amp, bool NT, bool SCATTER>
__global__ void __launch_bounds__(256) k_calib_rmw(Amp *__restrict__ p, int nbits, int cbits, double c, double s,
                                                   uint64_t i0)
{
    const uint64_t i = i0 + (uint64_t)blockIdx.x * 256u + threadIdx.x;
    uint64_t a = i;
    if (SCATTER) {
        const int hb = nbits - cbits;
        const uint64_t hi = i >> cbits, lo = i & ((1ull << cbits) - 1);
        a = (hb > 0 ? (__brevll(hi) >> (64 - hb)) << cbits : 0) | lo;
    }
    const double2 v = ld_amp(p + a, NT);
    st_amp(p + a, make_double2(c * v.x - s * v.y, c * v.y + s * v.x), NT);
}

template <typename Amp>
cfh_status launch_calib(Amp *p, int n, int cbits, bool nt, hipStream_t st)
{
    const double c = std::cos(0.25), s = std::sin(0.25);
    // one thread per amplitude, in launches of at most 2^31 threads (a launch
    // holds fewer than 2^32 work-items)
    const uint64_t N = 1ull << n, per = 1ull << 31;
    const bool sc = cbits >= 0;
    for (uint64_t i0 = 0; i0 < N; i0 += per) {
        const unsigned grid = (unsigned)(std::min(per, N - i0) / 256);
        if (nt && sc)
            hipLaunchKernelGGL((k_calib_rmw<Amp, true, true>), dim3(grid), dim3(256), 0, st, p, n, cbits, c, s, i0);
        else if (nt)
            hipLaunchKernelGGL((k_calib_rmw<Amp, true, false>), dim3(grid), dim3(256), 0, st, p, n, 0, c, s, i0);
        else if (sc)
            hipLaunchKernelGGL((k_calib_rmw<Amp, false, true>), dim3(grid), dim3(256), 0, st, p, n, cbits, c, s, i0);
        else
            hipLaunchKernelGGL((k_calib_rmw<Amp, false, false>), dim3(grid), dim3(256), 0, st, p, n, 0, c, s, i0);
        const cfh_status r = last_launch("k_calib_rmw");
        if (r) return r;
    }
    return CFH_OK;
}

} // namespace

extern "C" cfh_status cfh_calib_rmw(void *buf, int n, int dtype, int chunk_bits, int nontemporal, void *stream)
{
    if (!buf) return set_error(CFH_E_INVAL, "cfh_calib_rmw: null buffer");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_calib_rmw: dtype");
    if (n < 8 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_calib_rmw: n outside 8..34");
    if (chunk_bits < -1 || chunk_bits > n) return set_error(CFH_E_INVAL, "cfh_calib_rmw: chunk_bits outside -1..n");
    if (nontemporal != 0 && nontemporal != 1) return set_error(CFH_E_INVAL, "cfh_calib_rmw: nontemporal is 0 or 1");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == CFH_C128) return launch_calib((double2 *)buf, n, chunk_bits, nontemporal == 1, s);
    return launch_calib((float2 *)buf, n, chunk_bits, nontemporal == 1, s);
}
