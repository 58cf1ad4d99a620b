// <psi| H |psi> for a weighted Pauli sum without any allocation at call
// time: the per-workgroup partial sums live in a fixed device array of this
// translation unit instead of a buffer from cfh_ham_create.  Each term is
// evaluated by its definition (Eq. chfsexp with the action of a Pauli on
// basis states, Sec. 3): sum_y conj(psi_y) i^{(e - |x&z|) mod 4}
// (-1)^{|y&z|} psi_{y^x}, one read of the state per term.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "cfh_internal.hpp"
#include "device_common.hpp"
#include "launch.hpp"

using namespace cfh;
using namespace cfh::dev;

namespace {

constexpr unsigned kNaSlots = 2048;        // workgroups per launch at most = partial slots
constexpr int kNaThreads = 256;
constexpr int kNaTermsPerLaunch = 64;      // terms carried as kernel arguments
constexpr int kNaMaxDevices = 64;

// Partial sums of one call, one slot per workgroup.  Every call on a device
// uses that device's copy: calls that overlap in time on one device race.
static __device__ __align__(256) double2 scratch[kNaSlots];

struct NaTerm {
    uint64_t x, z;
    double wre, wim;  // coeff * i^{(e - |x&z|) mod 4}
};
struct NaTerms {
    NaTerm t[kNaTermsPerLaunch];
    int32_t count;
    int32_t first;  // 1: write the slots (first launch of a call), 0: add to them
};

template <typename Amp>
__global__ void __launch_bounds__(kNaThreads)
k_na_expval(const Amp *__restrict__ psi, uint64_t N, const NaTerms T, double2 *__restrict__ part)
{
    __shared__ double shr[kNaThreads], shi[kNaThreads];
    const uint64_t stride = (uint64_t)gridDim.x * kNaThreads;
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < T.count; ++k) {
        const uint64_t x = T.t[k].x, z = T.t[k].z;
        double sr = 0.0, si = 0.0;
        for (uint64_t y = (uint64_t)blockIdx.x * kNaThreads + threadIdx.x; y < N; y += stride) {
            const double2 a = ld(psi[y]), b = ld(psi[y ^ x]);
            const double pr = a.x * b.x + a.y * b.y, pi = a.x * b.y - a.y * b.x;  // conj(a) b
            if (par64(y & z)) {
                sr -= pr;
                si -= pi;
            } else {
                sr += pr;
                si += pi;
            }
        }
        ar += T.t[k].wre * sr - T.t[k].wim * si;
        ai += T.t[k].wre * si + T.t[k].wim * sr;
    }
    const int t = threadIdx.x;
    shr[t] = ar;
    shi[t] = ai;
    __syncthreads();
    for (int h = kNaThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            shr[t] += shr[t + h];
            shi[t] += shi[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double2 v = make_double2(shr[0], shi[0]);
        part[blockIdx.x] = T.first ? v : make_double2(part[blockIdx.x].x + v.x, part[blockIdx.x].y + v.y);
    }
}

// out[0] + i out[1] = sum of the cnt slots, in a fixed order.
__global__ void __launch_bounds__(kNaThreads) k_na_reduce(const double2 *__restrict__ part, int cnt,
                                                          double *__restrict__ out)
{
    __shared__ double shr[kNaThreads], shi[kNaThreads];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = t; i < cnt; i += kNaThreads) {
        a += part[i].x;
        b += part[i].y;
    }
    shr[t] = a;
    shi[t] = b;
    __syncthreads();
    for (int h = kNaThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            shr[t] += shr[t + h];
            shi[t] += shi[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = shr[0];
        out[1] = shi[0];
    }
}

std::mutex g_na_mutex;
double2 *g_na_slots[kNaMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  The array's name in host code is not a
// device address; only the looked-up pointer is passed to kernels.
cfh_status na_slots(double2 **out)
{
    int dev = -1;
    cfh_status st = CFH_OK;
    if (!hip_ok(hipGetDevice(&dev), "cfh_expval_noalloc: hipGetDevice", &st)) return st;
    if (dev < 0 || dev >= kNaMaxDevices) return set_error(CFH_E_UNSUPPORTED, "cfh_expval_noalloc: device index");
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_slots[dev]) {
        void *p = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "cfh_expval_noalloc: hipGetSymbolAddress", &st))
            return st;
        g_na_slots[dev] = static_cast<double2 *>(p);
    }
    *out = g_na_slots[dev];
    return CFH_OK;
}

template <typename Amp>
cfh_status na_run(const Amp *psi, int n, const cfh_pauli *terms, const double *coeff, size_t m, double *out_dev,
                  double2 *slots, hipStream_t s)
{
    const uint64_t N = 1ull << n;
    // about four amplitudes per thread per term, at most kNaSlots workgroups
    const uint64_t want = (N + 4ull * kNaThreads - 1) / (4ull * kNaThreads);
    const unsigned grid = (unsigned)(want < kNaSlots ? (want ? want : 1) : kNaSlots);
    if (grid > kNaSlots) return set_error(CFH_E_UNSUPPORTED, "cfh_expval_noalloc: more workgroups than slots");
    NaTerms T;
    size_t done = 0;
    bool first = true;
    do {
        const size_t cnt = std::min<size_t>(kNaTermsPerLaunch, m - done);
        for (size_t k = 0; k < cnt; ++k) {
            const cfh_pauli &p = terms[done + k];
            const int wp = (p.e - popc(p.x & p.z)) & 3;  // i^wp
            const double c = coeff[done + k];
            T.t[k].x = p.x;
            T.t[k].z = p.z;
            T.t[k].wre = wp == 0 ? c : wp == 2 ? -c : 0.0;
            T.t[k].wim = wp == 1 ? c : wp == 3 ? -c : 0.0;
        }
        T.count = (int32_t)cnt;
        T.first = first ? 1 : 0;
        hipLaunchKernelGGL((k_na_expval<Amp>), dim3(grid), dim3(kNaThreads), 0, s, psi, N, T, slots);
        const cfh_status st = last_launch("k_na_expval");
        if (st) return st;
        done += cnt;
        first = false;
    } while (done < m);
    hipLaunchKernelGGL(k_na_reduce, dim3(1), dim3(kNaThreads), 0, s, slots, (int)grid, out_dev);
    return last_launch("k_na_reduce");
}

} // namespace

extern "C" cfh_status cfh_expval_noalloc(const void *psi, int n, int dtype, const cfh_pauli *terms,
                                         const double *coeff, size_t m, double *out_dev, void *stream)
{
    if (!psi || !out_dev) return set_error(CFH_E_INVAL, "cfh_expval_noalloc: null state or output");
    if (m && (!terms || !coeff)) return set_error(CFH_E_INVAL, "cfh_expval_noalloc: null terms or coefficients");
    if (n < 1 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_expval_noalloc: n outside 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_expval_noalloc: dtype");
    for (size_t k = 0; k < m; ++k) {
        const cfh_status st = check_pauli(terms[k], n, true, "cfh_expval_noalloc");
        if (st) return st;
    }
    double2 *slots = nullptr;
    const cfh_status st = na_slots(&slots);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == CFH_C128)
        return na_run(static_cast<const double2 *>(psi), n, terms, coeff, m, out_dev, slots, s);
    return na_run(static_cast<const float2 *>(psi), n, terms, coeff, m, out_dev, slots, s);
}
