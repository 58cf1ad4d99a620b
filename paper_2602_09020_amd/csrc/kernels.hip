// gfx950 kernels of libcfh and the C-ABI entry points that launch them.
//
// The hot loop is the multi-qubit Pauli rotation of Sec. 3 applied to Phi
// (Sec. 4.2): amplitudes pair as (y, y ^ x) and each member of a pair gets the
// sign (-1)^{|y & z|}; App. B gives the 2x2 pair rule.  All kernels stream
// the state through HBM with 16-byte (c128) or 8-byte (c64) accesses;
// arithmetic is double precision in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <thread>
#include <tuple>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "cfh_internal.hpp"
#include "device_common.hpp"
#include "launch.hpp"

using namespace cfh;

namespace cfh {

bool hip_ok(hipError_t e, const char *what, cfh_status *st)
{
    if (e == hipSuccess) return true;
    *st = set_error(CFH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

cfh_status last_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CFH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return CFH_OK;
}

// Persistent grid: as many workgroups as can be resident at once (cached per
// kernel, LDS size and device).
unsigned resident_grid(const void *fn, int threads, size_t lds)
{
    // one cache for every thread that launches (the lock is uncontended after
    // each kernel's first launch)
    static std::mutex mu;
    static std::map<std::tuple<const void *, size_t, int>, unsigned> cache;
    std::lock_guard<std::mutex> lock(mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_tuple(fn, lds, dev);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    const unsigned g = (unsigned)(per_cu * cus);
    cache[key] = g;
    return g;
}

} // namespace cfh

namespace {

using namespace cfh::dev;

constexpr int threads_for(int B) { return B - 1 >= 8 ? 256 : (1 << (B - 1)); }
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// ------------------------------------------------------------ small kernels

__global__ void k_coef(const double *__restrict__ theta, double2 *__restrict__ coef, int64_t m)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        double s, c;
        sincos(0.5 * theta[k], &s, &c);
        coef[k] = make_double2(c, s);
    }
}

template <typename Amp>
__global__ void k_set_basis(Amp *__restrict__ psi, uint64_t N, uint64_t index)
{
    for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < N;
         y += (uint64_t)gridDim.x * blockDim.x)
        st(psi[y], make_double2(y == index ? 1.0 : 0.0, 0.0));
}

__global__ void k_zero_d(double *__restrict__ p, int64_t cnt)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// ---------------------------------------------- unfused rotation (one pass)
// Pair q -> y0 = q with a zero inserted at bit hb (the top bit of x), y1 = y0 ^ x.
// Consecutive lanes take consecutive q, so both members stream contiguously.
constexpr int kR1Threads = 256;
constexpr int kR1Pairs = 4;
// A launch holds fewer than 2^32 work-items; the single-rotation kernels loop
// over chunks, so one launch of at most this many workgroups covers any state.
constexpr uint64_t kR1MaxGrid = 1ull << 20;

template <typename Amp>
__global__ void __launch_bounds__(kR1Threads)
k_rot_pairs(Amp *__restrict__ psi, uint64_t x, uint64_t z, int hb, int w, int dsign, double c_in,
            double s_in, const double2 *__restrict__ coef, int k, double ssign, uint64_t npairs)
{
    double c = c_in, s = s_in;
    if (coef) {
        const double2 cs = coef[k];
        c = cs.x;
        s = cs.y * ssign;
    }
    const double sr = (w & 2) ? -s : s;
    const bool imag = w & 1;
    const uint64_t lowm = (1ull << hb) - 1;
    constexpr uint64_t per = (uint64_t)kR1Threads * kR1Pairs;
    for (uint64_t q0 = (uint64_t)blockIdx.x * per + threadIdx.x; q0 - threadIdx.x < npairs;
         q0 += (uint64_t)gridDim.x * per) {
        double2 u[kR1Pairs], v[kR1Pairs];
        uint64_t ya[kR1Pairs];
#pragma unroll
        for (int j = 0; j < kR1Pairs; ++j) {
            const uint64_t q = q0 + (uint64_t)j * kR1Threads;
            ya[j] = ((q & ~lowm) << 1) | (q & lowm);
            if (q < npairs) {
                u[j] = ld(psi[ya[j]]);
                v[j] = ld(psi[ya[j] ^ x]);
            }
        }
#pragma unroll
        for (int j = 0; j < kR1Pairs; ++j) {
            const uint64_t q = q0 + (uint64_t)j * kR1Threads;
            if (q < npairs) {
                const int sg0 = par64(ya[j] & z);
                const double s0 = sg0 ? -sr : sr;
                const double s1 = (sg0 ^ dsign) ? -sr : sr;
                rot_pair(u[j], v[j], c, s0, s1, imag);
                st(psi[ya[j]], u[j]);
                st(psi[ya[j] ^ x], v[j]);
            }
        }
    }
}

template <typename Amp>
__global__ void __launch_bounds__(kR1Threads)
k_rot_diag(Amp *__restrict__ psi, uint64_t z, int w, double c_in, double s_in,
           const double2 *__restrict__ coef, int k, double ssign, uint64_t N)
{
    double c = c_in, s = s_in;
    if (coef) {
        const double2 cs = coef[k];
        c = cs.x;
        s = cs.y * ssign;
    }
    const double sr = (w & 2) ? -s : s;
    const bool imag = w & 1;
    constexpr uint64_t per = (uint64_t)kR1Threads * kR1Pairs;
    for (uint64_t y0 = (uint64_t)blockIdx.x * per + threadIdx.x; y0 - threadIdx.x < N;
         y0 += (uint64_t)gridDim.x * per) {
#pragma unroll
        for (int j = 0; j < kR1Pairs; ++j) {
            const uint64_t y = y0 + (uint64_t)j * kR1Threads;
            if (y < N) {
                const double sj = par64(y & z) ? -sr : sr;
                st(psi[y], rot_diag(ld(psi[y]), c, sj, imag));
            }
        }
    }
}

// -------------------------------------------------- fused LDS tile pass
// One workgroup per coset base + V (see PassArgs).  Load the 2^B amplitudes of
// the coset (coalesced: the low local bits are unit vectors of the low index
// bits), apply the run of rotations in LDS, store once.
template <typename Amp, int B>
__global__ void __launch_bounds__(threads_for(B))
k_pass(Amp *__restrict__ psi, const double2 *__restrict__ coef, const PassArgs args)
{
    constexpr int T = threads_for(B);
    constexpr int LT = ilog2c(T);
    constexpr int N = 1 << B;
    constexpr int E = N / T;
    constexpr int NP = N / 2 / T;
    __shared__ Amp tile[N];
    const int t = threadIdx.x;
    const uint64_t base = deposit((uint64_t)blockIdx.x + (uint64_t)args.tile_base, args.outer_mask);
    uint64_t Lt = 0;
#pragma unroll
    for (int i = 0; i < LT; ++i)
        if ((t >> i) & 1) Lt ^= args.v[i];
    const uint64_t yb = base ^ Lt;
    Amp r[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        uint64_t Lk = 0;
#pragma unroll
        for (int i = 0; i < B - LT; ++i)
            if ((k >> i) & 1) Lk ^= args.v[LT + i];
        r[k] = psi[yb ^ Lk];
    }
#pragma unroll
    for (int k = 0; k < E; ++k) tile[t + k * T] = r[k];
    __syncthreads();

    for (int ri = 0; ri < args.nrot; ++ri) {
        const RotDesc &d = args.rot[args.inverse ? args.nrot - 1 - ri : ri];
        const double2 cs = coef[d.k];
        const double c = cs.x;
        double sr = args.inverse ? -cs.y : cs.y;
        if (d.w & 2) sr = -sr;
        const bool imag = d.w & 1;
        const int so = par64(base & d.z);
        if (d.xl == 0) {
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int a = t + k * T;
                const double sj = (par32(a & d.zl) ^ so) ? -sr : sr;
                st(tile[a], rot_diag(ld(tile[a]), c, sj, imag));
            }
        } else {
            const uint32_t lowm = (1u << d.hb) - 1;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const uint32_t q = t + k * T;
                const uint32_t a0 = ((q & ~lowm) << 1) | (q & lowm);
                const uint32_t a1 = a0 ^ d.xl;
                const int sg0 = par32(a0 & d.zl) ^ so;
                const double s0 = sg0 ? -sr : sr;
                const double s1 = (sg0 ^ d.dsign) ? -sr : sr;
                double2 u = ld(tile[a0]), v = ld(tile[a1]);
                rot_pair(u, v, c, s0, s1, imag);
                st(tile[a0], u);
                st(tile[a1], v);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < E; ++k) r[k] = tile[t + k * T];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        uint64_t Lk = 0;
#pragma unroll
        for (int i = 0; i < B - LT; ++i)
            if ((k >> i) & 1) Lk ^= args.v[LT + i];
        psi[yb ^ Lk] = r[k];
    }
}

// ------------------------------------------------ wave/block reductions

// ------------------------------------------------ Hamiltonian passes
// Read-only pass over cosets of a unit-vector subspace T (the qubits of the
// pass).  For each x-group with x inside T and each of its terms j:
//   sum_a conj(Phi[a]) * w_j * (-1)^{|y_a & z_j|} * Phi[a ^ xl],
// w_j = coeff_j * i^{(e_j - |x&z_j|) mod 4}  (Eq. chfsexp with the pair rule).
template <typename Amp, int B>
__global__ void __launch_bounds__(threads_for(B))
k_ham_expval(const Amp *__restrict__ psi, const HamPassArgs args, const HamGroupDev *__restrict__ groups,
             const HamTermDev *__restrict__ terms, double2 *__restrict__ partial, uint64_t ntiles)
{
    constexpr int T = threads_for(B);
    constexpr int LT = ilog2c(T);
    constexpr int N = 1 << B;
    constexpr int E = N / T;
    constexpr int W = (T + 63) / 64;
    __shared__ Amp tile[N];
    __shared__ double red[2][W];
    const int t = threadIdx.x;
    uint64_t Lt = 0;
#pragma unroll
    for (int i = 0; i < LT; ++i)
        if ((t >> i) & 1) Lt ^= args.v[i];
    double accr = 0.0, acci = 0.0;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint64_t base = deposit(tl, args.outer_mask);
        const uint64_t yb = base ^ Lt;
        Amp r[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            uint64_t Lk = 0;
#pragma unroll
            for (int i = 0; i < B - LT; ++i)
                if ((k >> i) & 1) Lk ^= args.v[LT + i];
            r[k] = psi[yb ^ Lk];
        }
#pragma unroll
        for (int k = 0; k < E; ++k) tile[t + k * T] = r[k];
        __syncthreads();
        for (int g = args.group_begin; g < args.group_begin + args.group_count; ++g) {
            const HamGroupDev G = groups[g];
            double pr[E], pi[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int a = t + k * T;
                const double2 u = ld(r[k]), v = ld(tile[a ^ G.xl]);
                pr[k] = u.x * v.x + u.y * v.y;   // conj(u) * v
                pi[k] = u.x * v.y - u.y * v.x;
            }
            for (int j = G.term_begin; j < G.term_begin + G.term_count; ++j) {
                const HamTermDev tm = terms[j];
                const int so = par64(base & tm.z);
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int a = t + k * T;
                    const double sg = (par32(a & tm.zl) ^ so) ? -1.0 : 1.0;
                    accr += sg * (tm.wre * pr[k] - tm.wim * pi[k]);
                    acci += sg * (tm.wre * pi[k] + tm.wim * pr[k]);
                }
            }
        }
        __syncthreads();
    }
    accr = wave_sum<(T < 64 ? T : 64)>(accr);
    acci = wave_sum<(T < 64 ? T : 64)>(acci);
    if ((t & 63) == 0) {
        red[0][t >> 6] = accr;
        red[1][t >> 6] = acci;
    }
    __syncthreads();
    if (t == 0) {
        double sr = 0, si = 0;
        for (int i = 0; i < W; ++i) {
            sr += red[0][i];
            si += red[1][i];
        }
        partial[blockIdx.x].x += sr;   // same block index -> same tiles in every pass
        partial[blockIdx.x].y += si;
    }
}

// out[y] (+)= sum_groups sum_terms w_j (-1)^{|y & z_j|} psi[y ^ x]  (H psi).
template <typename Amp, int B>
__global__ void __launch_bounds__(threads_for(B))
k_ham_apply(const Amp *__restrict__ psi, Amp *__restrict__ out, const HamPassArgs args,
            const HamGroupDev *__restrict__ groups, const HamTermDev *__restrict__ terms, int accumulate,
            uint64_t tile0)
{
    constexpr int T = threads_for(B);
    constexpr int LT = ilog2c(T);
    constexpr int N = 1 << B;
    constexpr int E = N / T;
    __shared__ Amp tile[N];
    const int t = threadIdx.x;
    const uint64_t base = deposit((uint64_t)blockIdx.x + tile0, args.outer_mask);
    uint64_t Lt = 0;
#pragma unroll
    for (int i = 0; i < LT; ++i)
        if ((t >> i) & 1) Lt ^= args.v[i];
    const uint64_t yb = base ^ Lt;
    uint64_t yk[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        uint64_t Lk = 0;
#pragma unroll
        for (int i = 0; i < B - LT; ++i)
            if ((k >> i) & 1) Lk ^= args.v[LT + i];
        yk[k] = yb ^ Lk;
        tile[t + k * T] = psi[yk[k]];
    }
    __syncthreads();
    double ar[E], ai[E];
#pragma unroll
    for (int k = 0; k < E; ++k) ar[k] = ai[k] = 0.0;
    for (int g = args.group_begin; g < args.group_begin + args.group_count; ++g) {
        const HamGroupDev G = groups[g];
        double vr[E], vi[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const double2 v = ld(tile[(t + k * T) ^ G.xl]);
            vr[k] = v.x;
            vi[k] = v.y;
        }
        for (int j = G.term_begin; j < G.term_begin + G.term_count; ++j) {
            const HamTermDev tm = terms[j];
            const int so = par64(base & tm.z);
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int a = t + k * T;
                const double sg = (par32(a & tm.zl) ^ so) ? -1.0 : 1.0;
                ar[k] += sg * (tm.wre * vr[k] - tm.wim * vi[k]);
                ai[k] += sg * (tm.wre * vi[k] + tm.wim * vr[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        double2 o = make_double2(ar[k], ai[k]);
        if (accumulate) {
            const double2 p = ld(out[yk[k]]);
            o.x += p.x;
            o.y += p.y;
        }
        st(out[yk[k]], o);
    }
}

__global__ void k_reduce_partial(const double2 *__restrict__ partial, int cnt, double *__restrict__ out)
{
    __shared__ double sr[256], si[256];
    const int t = threadIdx.x;
    double a = 0, b = 0;
    for (int i = t; i < cnt; i += 256) {
        a += partial[i].x;
        b += partial[i].y;
    }
    sr[t] = a;
    si[t] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sr[t] += sr[t + s];
            si[t] += si[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sr[0];
        out[1] = si[0];
    }
}

// ------------------------------------------------------ adjoint pass
// Tiles of psi and lam share LDS.  Walking the run backwards, rotation k
// contributes g_k = Im <lam| P_k |psi> on the coset and then both tiles are
// rewound by R_k^dag.  Per-wave partial sums live in LDS and are combined in
// a fixed order, so the result is bitwise reproducible.
template <typename Amp, int B>
__global__ void __launch_bounds__(threads_for(B))
k_adjoint_pass(Amp *__restrict__ psi, Amp *__restrict__ lam, const double2 *__restrict__ coef,
               const PassArgs args, double *__restrict__ partial, uint64_t ntiles)
{
    constexpr int T = threads_for(B);
    constexpr int LT = ilog2c(T);
    constexpr int N = 1 << B;
    constexpr int E = N / T;
    constexpr int NP = N / 2 / T;
    constexpr int W = (T + 63) / 64;
    __shared__ Amp tp[N];
    __shared__ Amp tl[N];
    __shared__ double wacc[kMaxRun][W];
    const int t = threadIdx.x;
    for (int i = t; i < kMaxRun * W; i += T) (&wacc[0][0])[i] = 0.0;
    uint64_t Lt = 0;
#pragma unroll
    for (int i = 0; i < LT; ++i)
        if ((t >> i) & 1) Lt ^= args.v[i];
    __syncthreads();
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t base = deposit(tile, args.outer_mask);
        const uint64_t yb = base ^ Lt;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            uint64_t Lk = 0;
#pragma unroll
            for (int i = 0; i < B - LT; ++i)
                if ((k >> i) & 1) Lk ^= args.v[LT + i];
            tp[t + k * T] = psi[yb ^ Lk];
            tl[t + k * T] = lam[yb ^ Lk];
        }
        __syncthreads();
        for (int ri = args.nrot - 1; ri >= 0; --ri) {
            const RotDesc &d = args.rot[ri];
            const double2 cs = coef[d.k];
            const double c = cs.x;
            double sr = -cs.y;             // R^dag: negated angle
            if (d.w & 2) sr = -sr;
            const bool imag = d.w & 1;
            const int wp = (d.w + 1) & 3;  // P psi carries i^{(e - |x&z|)}
            const int so = par64(base & d.z);
            double g = 0.0;
            if (d.xl == 0) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int a = t + k * T;
                    const int sg = par32(a & d.zl) ^ so;
                    const double2 u = ld(tp[a]), l = ld(tl[a]);
                    const double zr = l.x * u.x + l.y * u.y, zi = l.x * u.y - l.y * u.x;
                    const double im = (wp & 1) ? zr : zi;
                    g += ((wp & 2) ? -im : im) * (sg ? -1.0 : 1.0);
                    const double sj = sg ? -sr : sr;
                    st(tp[a], rot_diag(u, c, sj, imag));
                    st(tl[a], rot_diag(l, c, sj, imag));
                }
            } else {
                const uint32_t lowm = (1u << d.hb) - 1;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const uint32_t q = t + k * T;
                    const uint32_t a0 = ((q & ~lowm) << 1) | (q & lowm);
                    const uint32_t a1 = a0 ^ d.xl;
                    const int sg0 = par32(a0 & d.zl) ^ so;
                    const int sg1 = sg0 ^ d.dsign;
                    double2 u0 = ld(tp[a0]), u1 = ld(tp[a1]);
                    double2 l0 = ld(tl[a0]), l1 = ld(tl[a1]);
                    // conj(l0) (P psi)[a0] + conj(l1) (P psi)[a1], (P psi)[a0] ~ psi[a1]
                    const double z0r = l0.x * u1.x + l0.y * u1.y, z0i = l0.x * u1.y - l0.y * u1.x;
                    const double z1r = l1.x * u0.x + l1.y * u0.y, z1i = l1.x * u0.y - l1.y * u0.x;
                    const double zr = (sg0 ? -z0r : z0r) + (sg1 ? -z1r : z1r);
                    const double zi = (sg0 ? -z0i : z0i) + (sg1 ? -z1i : z1i);
                    const double im = (wp & 1) ? zr : zi;
                    g += (wp & 2) ? -im : im;
                    const double s0 = sg0 ? -sr : sr, s1 = sg1 ? -sr : sr;
                    rot_pair(u0, u1, c, s0, s1, imag);
                    rot_pair(l0, l1, c, s0, s1, imag);
                    st(tp[a0], u0);
                    st(tp[a1], u1);
                    st(tl[a0], l0);
                    st(tl[a1], l1);
                }
            }
            g = wave_sum<(T < 64 ? T : 64)>(g);
            if ((t & 63) == 0) wacc[ri][t >> 6] += g;
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            uint64_t Lk = 0;
#pragma unroll
            for (int i = 0; i < B - LT; ++i)
                if ((k >> i) & 1) Lk ^= args.v[LT + i];
            psi[yb ^ Lk] = tp[t + k * T];
            lam[yb ^ Lk] = tl[t + k * T];
        }
        __syncthreads();
    }
    if (t < args.nrot) {
        double s = 0.0;
        for (int i = 0; i < W; ++i) s += wacc[t][i];
        partial[(uint64_t)blockIdx.x * kMaxRun + t] = s;
    }
}

__global__ void k_grad_reduce(const double *__restrict__ partial, int nblocks, const PassArgs args,
                              double *__restrict__ grad)
{
    const int ri = blockIdx.x;
    __shared__ double s[256];
    double a = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) a += partial[(uint64_t)b * kMaxRun + ri];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[args.rot[ri].k] = s[0];
}

// ------------------------------------------------------ device frame map
// One thread per string; the 2n frame rows are staged in LDS.
struct FrameRowDev {
    uint64_t x, z;
    int32_t e, pad;
};

__device__ __forceinline__ void dmul(uint64_t &x, uint64_t &z, int &e, uint64_t bx, uint64_t bz, int be)
{
    const uint64_t rx = x ^ bx, rz = z ^ bz;
    e = (e + be + __builtin_popcountll(x & z) + __builtin_popcountll(bx & bz) +
         2 * __builtin_popcountll(z & bx) - __builtin_popcountll(rx & rz)) & 3;
    x = rx;
    z = rz;
}

__global__ void k_frame_conjugate(const FrameRowDev *__restrict__ rows, int n, const cfh_pauli *__restrict__ in,
                                  cfh_pauli *__restrict__ out, uint64_t m)
{
    __shared__ FrameRowDev s[2 * kMaxFrameQubits];
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) s[i] = rows[i];
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const cfh_pauli p = in[i];
    uint64_t x = 0, z = 0;
    int e = p.e & 3;
    uint64_t supp = p.x | p.z;
    while (supp) {
        const int j = __builtin_ctzll(supp);
        supp &= supp - 1;
        const bool xb = (p.x >> j) & 1, zb = (p.z >> j) & 1;
        const FrameRowDev &Z = s[j], &X = s[n + j];
        if (xb && zb) {           // i effX_j effZ_j
            uint64_t yx = X.x, yz = X.z;
            int ye = X.e;
            dmul(yx, yz, ye, Z.x, Z.z, Z.e);
            dmul(x, z, e, yx, yz, (ye + 1) & 3);
        } else if (xb) {
            dmul(x, z, e, X.x, X.z, X.e);
        } else {
            dmul(x, z, e, Z.x, Z.z, Z.e);
        }
    }
    out[i] = cfh_pauli{x, z, e, 0};
}

// ------------------------------------------------------ launch helpers
size_t amp_bytes(int dtype) { return dtype == CFH_C64 ? 8 : 16; }

template <typename Amp, int B>
constexpr bool fits_lds(int tiles) { return (size_t)tiles * sizeof(Amp) * ((size_t)1 << B) <= 160 * 1024; }

template <typename Amp>
cfh_status launch_pass(int b, uint64_t ntiles, hipStream_t s, Amp *psi, const double2 *coef, PassArgs a)
{
    // A launch holds fewer than 2^32 work-items: small tiles of a large state
    // (2^(n-b) workgroups of threads_for(b) threads) take several launches.
    if (b < 1 || b > 14) return set_error(CFH_E_UNSUPPORTED, "tile_bits outside 1..14");
    const uint64_t max_grid = (1ull << 31) / (uint64_t)threads_for(b);
    for (uint64_t off = 0; off < ntiles; off += max_grid) {
        a.tile_base = off;
        const unsigned g = (unsigned)std::min<uint64_t>(max_grid, ntiles - off);
        switch (b) {
#define CFH_PASS_CASE(BB)                                                                        \
    case BB:                                                                                     \
        if constexpr (fits_lds<Amp, BB>(1))                                                      \
            hipLaunchKernelGGL((k_pass<Amp, BB>), dim3(g), dim3(threads_for(BB)), 0, s, psi, coef, a); \
        else                                                                                     \
            return set_error(CFH_E_UNSUPPORTED, "tile_bits too large for LDS");                  \
        break;
            CFH_PASS_CASE(1) CFH_PASS_CASE(2) CFH_PASS_CASE(3) CFH_PASS_CASE(4) CFH_PASS_CASE(5)
            CFH_PASS_CASE(6) CFH_PASS_CASE(7) CFH_PASS_CASE(8) CFH_PASS_CASE(9) CFH_PASS_CASE(10)
            CFH_PASS_CASE(11) CFH_PASS_CASE(12) CFH_PASS_CASE(13) CFH_PASS_CASE(14)
#undef CFH_PASS_CASE
        default:
            return set_error(CFH_E_UNSUPPORTED, "tile_bits outside 1..14");
        }
    }
    return last_launch("k_pass");
}


template <typename Amp>
cfh_status launch_ham(int b, uint64_t ntiles, unsigned grid, hipStream_t s, const Amp *psi, Amp *out,
                      const HamPassArgs &a, const HamGroupDev *gr, const HamTermDev *tm, double2 *partial,
                      int accumulate)
{
    switch (b) {
#define CFH_HAM_CASE(BB)                                                                                   \
    case BB:                                                                                               \
        if constexpr (fits_lds<Amp, BB>(1) && BB <= 13) {                                                  \
            if (out) {                                                                                     \
                /* fewer than 2^32 work-items per launch */                                                \
                constexpr uint64_t G = (1ull << 31) / threads_for(BB);                                     \
                for (uint64_t t0 = 0; t0 < ntiles; t0 += G)                                                \
                    hipLaunchKernelGGL((k_ham_apply<Amp, BB>), dim3((unsigned)std::min(G, ntiles - t0)),   \
                                       dim3(threads_for(BB)), 0, s, psi, out, a, gr, tm, accumulate, t0);  \
            } else                                                                                         \
                hipLaunchKernelGGL((k_ham_expval<Amp, BB>), dim3(grid), dim3(threads_for(BB)), 0, s, psi, a, \
                                   gr, tm, partial, ntiles);                                               \
        } else                                                                                             \
            return set_error(CFH_E_UNSUPPORTED, "tile_bits too large for LDS");                            \
        break;
        CFH_HAM_CASE(1) CFH_HAM_CASE(2) CFH_HAM_CASE(3) CFH_HAM_CASE(4) CFH_HAM_CASE(5)
        CFH_HAM_CASE(6) CFH_HAM_CASE(7) CFH_HAM_CASE(8) CFH_HAM_CASE(9) CFH_HAM_CASE(10)
        CFH_HAM_CASE(11) CFH_HAM_CASE(12) CFH_HAM_CASE(13) CFH_HAM_CASE(14)
#undef CFH_HAM_CASE
    default:
        return set_error(CFH_E_UNSUPPORTED, "tile_bits outside 1..14");
    }
    return last_launch("k_ham");
}

template <typename Amp>
cfh_status launch_adjoint(int b, uint64_t ntiles, unsigned grid, hipStream_t s, Amp *psi, Amp *lam,
                          const double2 *coef, const PassArgs &a, double *partial)
{
    switch (b) {
#define CFH_ADJ_CASE(BB)                                                                          \
    case BB:                                                                                      \
        if constexpr (fits_lds<Amp, BB>(2))                                                       \
            hipLaunchKernelGGL((k_adjoint_pass<Amp, BB>), dim3(grid), dim3(threads_for(BB)), 0, s, psi, lam, \
                               coef, a, partial, ntiles);                                         \
        else                                                                                      \
            return set_error(CFH_E_UNSUPPORTED, "tile_bits too large for the adjoint's two LDS tiles"); \
        break;
        CFH_ADJ_CASE(1) CFH_ADJ_CASE(2) CFH_ADJ_CASE(3) CFH_ADJ_CASE(4) CFH_ADJ_CASE(5)
        CFH_ADJ_CASE(6) CFH_ADJ_CASE(7) CFH_ADJ_CASE(8) CFH_ADJ_CASE(9) CFH_ADJ_CASE(10)
        CFH_ADJ_CASE(11) CFH_ADJ_CASE(12) CFH_ADJ_CASE(13)
#undef CFH_ADJ_CASE
    default:
        return set_error(CFH_E_UNSUPPORTED, "tile_bits outside 1..13 for the adjoint");
    }
    return last_launch("k_adjoint_pass");
}

cfh_status check_state_args(const void *psi, int n, int dtype, const char *what)
{
    if (!psi) return set_error(CFH_E_INVAL, std::string(what) + ": null state pointer");
    if (n < 1 || n > kMaxStateQubits)
        return set_error(CFH_E_UNSUPPORTED, std::string(what) + ": n must be in 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128)
        return set_error(CFH_E_UNSUPPORTED, std::string(what) + ": unknown dtype");
    return CFH_OK;
}

// psi_y <- c psi_y + s omega (-1)^{|y&z|} psi_{y^x} with omega = i^w,
// w = (e - |x&z| + wadd) mod 4: wadd = 3 is the rotation exp(-i theta/2 P)
// (omega = -i i^{e-|x&z|}, c = cos, s = sin of theta/2); wadd = 0 gives
// c psi + s P psi, the projector (1 + s P)/2 for c = s = 1/2.
template <typename Amp>
cfh_status rot_one(Amp *psi, int n, uint64_t x, uint64_t z, int e, double c, double s,
                   const double2 *coef, int k, double ssign, hipStream_t st, int wadd = 3)
{
    const int w = (e - popc(x & z) + wadd) & 3;
    const uint64_t per = (uint64_t)kR1Threads * kR1Pairs;
    if (x == 0) {
        const uint64_t N = 1ull << n;
        const unsigned g = (unsigned)std::min<uint64_t>((N + per - 1) / per, kR1MaxGrid);
        hipLaunchKernelGGL((k_rot_diag<Amp>), dim3(g), dim3(kR1Threads), 0, st, psi, z, w, c, s, coef, k, ssign, N);
        return last_launch("k_rot_diag");
    }
    const int hb = 63 - __builtin_clzll(x);
    const uint64_t np = 1ull << (n - 1);
    const unsigned g = (unsigned)std::min<uint64_t>((np + per - 1) / per, kR1MaxGrid);
    hipLaunchKernelGGL((k_rot_pairs<Amp>), dim3(g), dim3(kR1Threads), 0, st, psi, x, z, hb, w, popc(x & z) & 1, c,
                       s, coef, k, ssign, np);
    return last_launch("k_rot_pairs");
}

} // namespace

// ============================================================ plan object
struct cfh_plan_s {
    int n = 0, dtype = 0;
    TuningResolved tu{};
    std::vector<Pauli> rot;
    std::vector<PassPlan> passes;
    std::vector<PassArgs> args;
    bool v2 = false;                      // register-tiled kernel for the forward/inverse sweep
    int mode2 = 0;                        // k_pass2 MODE bits of the forward passes
    std::vector<PassArgs2> args2, args2_inv;
    double2 *coef = nullptr;     // device, m entries
    double *gpart = nullptr;     // device, adj_grid * kMaxRun
    unsigned adj_grid = 0;
    std::vector<PassArgs> adj_args;       // passes of the LDS-staged adjoint sweep (two LDS tiles)
    int adj_b = 0;
    std::vector<PassArgs2> adj2_args;     // register-tiled adjoint sweep: inverse-order descriptors
    static constexpr unsigned kAdj2Grid = 2048;
    ~cfh_plan_s()
    {
        if (coef) (void)hipFree(coef);
        if (gpart) (void)hipFree(gpart);
    }
};

struct cfh_ham_s {
    int n = 0, dtype = 0;
    TuningResolved tu{};
    std::vector<HamPass> passes;        // LDS-staged passes (H psi for the adjoint, small tiles)
    std::vector<HamPassArgs> args;
    HamGroupDev *groups = nullptr;
    HamTermDev *terms = nullptr;
    double2 *partial = nullptr;         // max(grid, kMeasureGrid) entries
    unsigned grid = 0;
    int64_t n_groups = 0;
    // register-tiled measurement passes for <H> (used when mmode != 0)
    std::vector<PassArgs2> margs;
    // register-tiled H psi passes (psi and lam in registers), when not empty
    std::vector<PassArgs2> hargs;
    double2 *mw = nullptr;              // per-term weight c_k i^{(e-|x&z|)}
    int mmode = 0;
    static constexpr unsigned kMeasureGrid = 2048;
    ~cfh_ham_s()
    {
        if (groups) (void)hipFree(groups);
        if (terms) (void)hipFree(terms);
        if (partial) (void)hipFree(partial);
        if (mw) (void)hipFree(mw);
    }
};

namespace {

// A planning task run on its own thread, or on the caller's if no thread can
// be started.  finish() joins it and returns its status, with its error
// message set again on the calling thread.  The destructor joins a task that
// was started and not finished (an early return), so no thread outlives the
// data it reads.
class PlanJob {
public:
    explicit PlanJob(std::function<cfh_status()> f) : f_(std::move(f)) {}
    ~PlanJob()
    {
        if (t_.joinable()) t_.join();
    }
    void start()
    {
        try {
            t_ = std::thread([this] { run(); });
        } catch (...) {
            run();
        }
    }
    cfh_status finish()
    {
        if (t_.joinable()) t_.join();
        return st_ ? set_error(st_, msg_) : CFH_OK;
    }

private:
    void run()
    {
        st_ = f_();
        if (st_) msg_ = cfh_last_error();
    }
    std::function<cfh_status()> f_;
    std::thread t_;
    cfh_status st_ = CFH_OK;
    std::string msg_;
};

unsigned persistent_grid(uint64_t ntiles)
{
    return (unsigned)std::min<uint64_t>(ntiles, 2048);
}

cfh_status build_pass_args(const std::vector<PassPlan> &passes, const std::vector<Pauli> &rot,
                           std::vector<PassArgs> &out)
{
    out.resize(passes.size());
    for (size_t i = 0; i < passes.size(); ++i) {
        const PassPlan &pp = passes[i];
        PassArgs &a = out[i];
        std::memset(&a, 0, sizeof(a));
        a.outer_mask = pp.outer_mask;
        for (int j = 0; j < pp.b; ++j) a.v[j] = pp.v[j];
        a.b = pp.b;
        a.nrot = (int)pp.rots.size();
        for (int j = 0; j < a.nrot; ++j) {
            const int k = pp.rots[j];
            bool in_span = false;
            local_coords(pp.v, rot[k].x, &in_span);
            if (!in_span) return set_error(CFH_E_INVAL, "planner produced a rotation outside its tile span");
            a.rot[j] = make_rot_desc(pp, rot[k], k);
        }
    }
    return CFH_OK;
}

} // namespace

extern "C" {

int cfh_device_count(void)
{
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) return 0;
    return c;
}

cfh_status cfh_state_set_basis(void *psi, int n, int dtype, uint64_t index, void *stream)
{
    cfh_status st = check_state_args(psi, n, dtype, "cfh_state_set_basis");
    if (st) return st;
    const uint64_t N = 1ull << n;
    if (index >= N) return set_error(CFH_E_RANGE, "cfh_state_set_basis: index >= 2^n");
    const unsigned grid = (unsigned)std::min<uint64_t>((N + 255) / 256, 1u << 20);
    if (dtype == CFH_C128)
        hipLaunchKernelGGL((k_set_basis<double2>), dim3(grid), dim3(256), 0, (hipStream_t)stream,
                           (double2 *)psi, N, index);
    else
        hipLaunchKernelGGL((k_set_basis<float2>), dim3(grid), dim3(256), 0, (hipStream_t)stream,
                           (float2 *)psi, N, index);
    return last_launch("k_set_basis");
}

cfh_status cfh_apply_pauli_rotation(void *psi, int n, int dtype, uint64_t x, uint64_t z, int e, double theta,
                                    void *stream)
{
    cfh_status st = check_state_args(psi, n, dtype, "cfh_apply_pauli_rotation");
    if (st) return st;
    st = check_pauli(cfh_pauli{x, z, e, 0}, n, true, "cfh_apply_pauli_rotation");
    if (st) return st;
    const double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
    if (dtype == CFH_C128)
        return rot_one((double2 *)psi, n, x, z, e, c, s, nullptr, 0, 1.0, (hipStream_t)stream);
    return rot_one((float2 *)psi, n, x, z, e, c, s, nullptr, 0, 1.0, (hipStream_t)stream);
}

cfh_status cfh_measure_pauli(void *psi, int n, int dtype, const cfh_pauli *p, double u, int32_t *outcome,
                             double *prob_plus, void *stream)
{
    cfh_status st = check_state_args(psi, n, dtype, "cfh_measure_pauli");
    if (st) return st;
    if (!p || !outcome) return set_error(CFH_E_INVAL, "cfh_measure_pauli: null argument");
    st = check_pauli(*p, n, true, "cfh_measure_pauli");
    if (st) return st;
    if (!(u >= 0.0 && u < 1.0)) return set_error(CFH_E_INVAL, "cfh_measure_pauli: u must be in [0, 1)");
    // P(+1) = (1 + <P>)/2; the outcome s is +1 when u < P(+1)
    const double one = 1.0;
    double ev[2] = {0.0, 0.0};
    st = cfh_expval(psi, n, dtype, p, &one, 1, ev, stream);
    if (st) return st;
    const double pp = std::min(1.0, std::max(0.0, 0.5 * (1.0 + ev[0])));
    const int sgn = u < pp ? 1 : -1;
    const double ps = sgn > 0 ? pp : 1.0 - pp;
    // collapse: psi <- (psi + s P psi) / (2 sqrt(P(s)))
    const double a = 0.5 / std::sqrt(ps);
    st = dtype == CFH_C128
             ? rot_one((double2 *)psi, n, p->x, p->z, p->e, a, sgn * a, nullptr, 0, 1.0, (hipStream_t)stream, 0)
             : rot_one((float2 *)psi, n, p->x, p->z, p->e, a, sgn * a, nullptr, 0, 1.0, (hipStream_t)stream, 0);
    if (st) return st;
    *outcome = sgn;
    if (prob_plus) *prob_plus = pp;
    return CFH_OK;
}

cfh_status cfh_plan_create(int n, int dtype, const cfh_pauli *rot, size_t m, const cfh_tuning *tuning,
                           cfh_plan *out)
{
    if (!out || (m && !rot)) return set_error(CFH_E_INVAL, "cfh_plan_create: null argument");
    if (n < 1 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_plan_create: n must be in 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_plan_create: dtype");
    if (m > (size_t)INT32_MAX) return set_error(CFH_E_INVAL, "cfh_plan_create: too many rotations");
    for (size_t i = 0; i < m; ++i) {
        cfh_status st = check_pauli(rot[i], n, true, "cfh_plan_create");
        if (st) return st;
    }
    std::unique_ptr<cfh_plan_s> p(new (std::nothrow) cfh_plan_s);
    if (!p) return set_error(CFH_E_NOMEM, "cfh_plan_create: host memory");
    p->n = n;
    p->dtype = dtype;
    p->tu = resolve_tuning(tuning, n, dtype, kTuneForward);
    if (tuning && (tuning->block_threads != 0 && tuning->block_threads != 256))
        return set_error(CFH_E_UNSUPPORTED, "cfh_plan_create: block_threads must be 256");
    p->rot.resize(m);
    for (size_t i = 0; i < m; ++i) p->rot[i] = Pauli{rot[i].x, rot[i].z, rot[i].e & 3};
    if (!p->tu.unfused) {
        p->passes = plan_rotations(n, p->rot, p->tu);
        const int b = p->tu.tile_bits;
        if (p->tu.variant < 0 || p->tu.variant > 5)
            return set_error(CFH_E_INVAL, "cfh_plan_create: unknown kernel variant");
        if (p->tu.variant >= 2 && p->tu.variant <= 4 && (b < 10 || b > 13))
            return set_error(CFH_E_UNSUPPORTED, "cfh_plan_create: the register-tiled kernel needs tile_bits in 10..13");
        if (p->tu.variant == 5 && (b < 10 || b > 14))
            return set_error(CFH_E_UNSUPPORTED, "cfh_plan_create: the half-tile kernel needs tile_bits in 10..14");
        // default: register-tiled with compile-time bodies where the tile
        // shape allows it (half-tile transposes for 2^14), LDS-staged otherwise
        int v = p->tu.variant;
        if (v == 0) v = b == 14 ? 5 : (b >= 10 && b <= 13) ? 4 : 1;
        p->tu.variant = v;
        // compile-time bodies in the tangent form (MODE bit 4), half-tile
        // transposes for variant 5
        p->mode2 = v == 2 ? 1 : v == 4 ? 18 : v == 5 ? 22 : 0;
        if (v >= 2) {
            // A run that needs more micro-groups than the kernel carries (long
            // runs of dense masks) is split in two on the same tile basis; the
            // halves keep the order of the run.
            std::vector<PassPlan> fitted;
            std::vector<PassPlan> todo(p->passes.rbegin(), p->passes.rend());
            PassArgs2 fa, ia;
            while (!todo.empty()) {
                PassPlan pp = std::move(todo.back());
                todo.pop_back();
                if (build_pass_args2(pp, p->rot, false, v == 5, fa) && build_pass_args2(pp, p->rot, true, v == 5, ia)) {
                    fitted.push_back(std::move(pp));
                    fa.xrot = ia.xrot = line_share_bits(fa.outer_mask, n, fa.b, (int)amp_bytes(dtype), p->tu.tile_order);
                    p->args2.push_back(fa);
                    p->args2_inv.push_back(ia);
                    continue;
                }
                if (pp.rots.size() < 2)
                    return set_error(CFH_E_INVAL, "cfh_plan_create: a rotation does not fit the register-tiled kernel");
                PassPlan hi = pp;
                const size_t half = pp.rots.size() / 2;
                hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
                pp.rots.resize(half);
                todo.push_back(std::move(hi));
                todo.push_back(std::move(pp));
            }
            p->passes = std::move(fitted);
            p->v2 = true;
        }
        cfh_status st = build_pass_args(p->passes, p->rot, p->args);
        if (st) return st;
    }
    // The adjoint sweep keeps a tile of the state and one of lam in LDS, so it
    // has its own pass list on tiles of at most 2^12 (c128) / 2^13 (c64).
    {
        TuningResolved ta = resolve_tuning(tuning, n, dtype, kTuneAdjoint);
        ta.unfused = 0;
        const int bcap = dtype == CFH_C128 ? 12 : 13;
        if (ta.tile_bits > bcap) ta.tile_bits = bcap;
        if (ta.tile_bits < n) ta.low_bits = std::min(ta.low_bits, ta.tile_bits - 1);
        if (!p->tu.unfused && ta.tile_bits == p->tu.tile_bits && ta.low_bits == p->tu.low_bits &&
            ta.max_run == p->tu.max_run && ta.lookahead == p->tu.lookahead) {
            p->adj_args = p->args;
        } else {
            cfh_status st = build_pass_args(plan_rotations(n, p->rot, ta), p->rot, p->adj_args);
            if (st) return st;
        }
        p->adj_b = ta.tile_bits;
    }
    // Register-tiled adjoint: psi and lam of a coset in registers, both moved
    // through LDS between micro-groups (half-tile transposes), so it has its
    // own pass list on 2^13 (c128) / 2^14 (c64) tiles.  Tuning variant 1
    // keeps the LDS-staged adjoint.
    if (p->tu.variant != 1 && !p->rot.empty()) {
        TuningResolved t2 = resolve_tuning(tuning, n, dtype, kTuneAdjoint2);
        // psi and lam of 16 amplitudes each per thread: at 2^14 the 1,024-thread
        // workgroups cannot hold them without spilling, so 2^13 at most
        t2.tile_bits = std::min(t2.tile_bits, 13);
        if (t2.tile_bits < n) t2.low_bits = std::min(t2.low_bits, t2.tile_bits - 1);
        if (t2.tile_bits >= 10 && t2.tile_bits <= 14) {
            t2.unfused = 0;
            std::vector<PassPlan> todo;
            for (PassPlan &pp : plan_rotations(n, p->rot, t2)) todo.push_back(std::move(pp));
            std::reverse(todo.begin(), todo.end());
            PassArgs2 ia;
            while (!todo.empty()) {
                PassPlan pp = std::move(todo.back());
                todo.pop_back();
                if (build_pass_args2(pp, p->rot, true, true, ia)) {
                    ia.xrot = line_share_bits(ia.outer_mask, n, ia.b, (int)amp_bytes(dtype), t2.tile_order);
                    p->adj2_args.push_back(ia);
                    continue;
                }
                if (pp.rots.size() < 2)
                    return set_error(CFH_E_INVAL, "cfh_plan_create: a rotation does not fit the adjoint kernel");
                PassPlan hi = pp;
                const size_t half = pp.rots.size() / 2;
                hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
                pp.rots.resize(half);
                todo.push_back(std::move(hi));
                todo.push_back(std::move(pp));
            }
        }
    }
    cfh_status st = CFH_OK;
    if (m && !hip_ok(hipMalloc(&p->coef, m * sizeof(double2)), "cfh_plan_create: hipMalloc", &st)) return st;
    // adjoint partial sums: one row of kMaxRun per persistent workgroup
    p->adj_grid = persistent_grid(1ull << (n - p->adj_b));
    const size_t gp = std::max<size_t>(p->adj_grid, p->adj2_args.empty() ? 0 : cfh_plan_s::kAdj2Grid);
    if (!hip_ok(hipMalloc(&p->gpart, gp * kMaxRun * sizeof(double)), "cfh_plan_create: hipMalloc", &st)) return st;
    *out = p.release();
    return CFH_OK;
}

cfh_status cfh_plan_destroy(cfh_plan p)
{
    delete p;
    return CFH_OK;
}

cfh_status cfh_plan_info(cfh_plan p, int64_t *n_passes, int64_t *n_rot, int32_t *tile_bits, double *hbm_bytes,
                         int32_t *variant)
{
    if (!p) return set_error(CFH_E_INVAL, "cfh_plan_info: null plan");
    const int64_t np = p->tu.unfused ? (int64_t)p->rot.size() : (int64_t)p->passes.size();
    if (n_passes) *n_passes = np;
    if (n_rot) *n_rot = (int64_t)p->rot.size();
    if (tile_bits) *tile_bits = p->tu.unfused ? 0 : p->tu.tile_bits;
    if (hbm_bytes) *hbm_bytes = 2.0 * (double)np * (double)(1ull << p->n) * (double)amp_bytes(p->dtype);
    if (variant) *variant = p->tu.unfused ? 0 : p->tu.variant;
    return CFH_OK;
}

cfh_status cfh_plan_schedule(cfh_plan p, int64_t *pass_start, int64_t *order)
{
    if (!p || !pass_start || !order) return set_error(CFH_E_INVAL, "cfh_plan_schedule: null argument");
    if (p->tu.unfused) {
        for (size_t i = 0; i <= p->rot.size(); ++i) pass_start[i] = (int64_t)i;
        for (size_t i = 0; i < p->rot.size(); ++i) order[i] = (int64_t)i;
        return CFH_OK;
    }
    int64_t o = 0;
    for (size_t i = 0; i < p->passes.size(); ++i) {
        pass_start[i] = o;
        for (int k : p->passes[i].rots) order[o++] = k;
    }
    pass_start[p->passes.size()] = o;
    return CFH_OK;
}

cfh_status cfh_plan_leaf_counts(cfh_plan p, const double *theta_host, int inverse, int64_t *counts)
{
    if (!p || !counts || (!theta_host && !p->rot.empty()))
        return set_error(CFH_E_INVAL, "cfh_plan_leaf_counts: null argument");
    if (p->tu.unfused || !(p->mode2 & 2) || p->args2.size() != p->passes.size())
        return set_error(CFH_E_UNSUPPORTED, "cfh_plan_leaf_counts: the plan does not run the compile-time bodies");
    std::fill(counts, counts + 512, (int64_t)0);
    const bool tanf = (p->mode2 & 16) != 0;
    for (const PassArgs2 &a : inverse ? p->args2_inv : p->args2) {
        const int nrot = a.mg[a.nmg - 1].rot_begin + a.mg[a.nmg - 1].rot_count;
        for (int ri = 0; ri < nrot; ++ri) {
            const RotDesc2 &d = a.rot[ri];
            const double th = theta_host[d.k];
            // the kernel's test on (cos, sin) of theta/2, which sign flips do not change
            const bool tan = tanf && std::fabs(std::sin(0.5 * th)) <= std::fabs(std::cos(0.5 * th));
            ++counts[(d.kase & 255u) | (tan ? 256u : 0u)];
        }
    }
    return CFH_OK;
}

cfh_status cfh_apply_plan(cfh_plan p, void *psi, const double *theta_dev, int inverse, void *stream)
{
    if (!p || !psi || (!theta_dev && !p->rot.empty())) return set_error(CFH_E_INVAL, "cfh_apply_plan: null argument");
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = (int64_t)p->rot.size();
    if (m == 0) return CFH_OK;
    hipLaunchKernelGGL(k_coef, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, theta_dev, p->coef, m);
    cfh_status st = last_launch("k_coef");
    if (st) return st;
    const double ssign = inverse ? -1.0 : 1.0;
    if (p->tu.unfused) {
        for (int64_t i = 0; i < m; ++i) {
            const int64_t k = inverse ? m - 1 - i : i;
            const Pauli &r = p->rot[k];
            st = p->dtype == CFH_C128
                     ? rot_one((double2 *)psi, p->n, r.x, r.z, r.e, 0, 0, p->coef, (int)k, ssign, s)
                     : rot_one((float2 *)psi, p->n, r.x, r.z, r.e, 0, 0, p->coef, (int)k, ssign, s);
            if (st) return st;
        }
        return CFH_OK;
    }
    const int64_t np = (int64_t)p->args.size();
    if (p->v2) {
        for (int64_t i = 0; i < np; ++i) {
            const PassArgs2 &a = inverse ? p->args2_inv[np - 1 - i] : p->args2[i];
            const uint64_t ntiles = 1ull << (p->n - a.b);
            st = p->dtype == CFH_C128 ? launch_pass2(ntiles, s, (double2 *)psi, p->coef, a, p->mode2)
                                      : launch_pass2(ntiles, s, (float2 *)psi, p->coef, a, p->mode2);
            if (st) return st;
        }
        return CFH_OK;
    }
    for (int64_t i = 0; i < np; ++i) {
        PassArgs a = p->args[inverse ? np - 1 - i : i];
        a.inverse = inverse ? 1 : 0;
        const uint64_t ntiles = 1ull << (p->n - a.b);
        st = p->dtype == CFH_C128 ? launch_pass(a.b, ntiles, s, (double2 *)psi, p->coef, a)
                                  : launch_pass(a.b, ntiles, s, (float2 *)psi, p->coef, a);
        if (st) return st;
    }
    return CFH_OK;
}

// ------------------------------------------------------------- Hamiltonians
cfh_status cfh_ham_create(int n, int dtype, const cfh_pauli *terms, const double *coeff, size_t m,
                          const cfh_tuning *tuning, cfh_ham *out)
{
    if (!out || (m && (!terms || !coeff))) return set_error(CFH_E_INVAL, "cfh_ham_create: null argument");
    if (n < 1 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_ham_create: n must be in 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_ham_create: dtype");
    for (size_t i = 0; i < m; ++i) {
        cfh_status st = check_pauli(terms[i], n, true, "cfh_ham_create");
        if (st) return st;
    }
    std::unique_ptr<cfh_ham_s> h(new (std::nothrow) cfh_ham_s);
    if (!h) return set_error(CFH_E_NOMEM, "cfh_ham_create: host memory");
    h->n = n;
    h->dtype = dtype;
    h->tu = resolve_tuning(tuning, n, dtype, kTuneHamiltonian);
    {
        // the LDS-staged passes (H psi, and <H> below 2^10) hold a whole tile
        // in LDS: 2^13 amplitudes at most (2^14 complex64 would fit LDS, but
        // its 1,024-thread workgroups cannot hold the kernel's registers)
        const int lcap = 13;
        if (h->tu.tile_bits > lcap) h->tu.tile_bits = lcap;
        if (h->tu.tile_bits < n) h->tu.low_bits = std::min(h->tu.low_bits, h->tu.tile_bits - 1);
    }
    const std::vector<HamGroup> groups = group_terms(terms, m);
    h->n_groups = (int64_t)groups.size();
    // The register-tiled term passes (<H>, and H psi for the adjoint) are
    // planned on two worker threads while this thread plans the LDS-staged
    // passes: the planners only read the groups and terms, and each writes
    // its own pass list.  A worker's error message is carried back to this
    // thread (the message store is per thread).
    //
    // <H> on the register-tiled kernel: passes of at most kMaxRun terms on
    // 2^b tiles (half-tile transposes at 2^14), terms ordered so consecutive
    // ones share register micro-groups.  The LDS-staged passes stay for H psi
    // and for tiles below 2^10.
    const MeasureSettings ms = measure_settings(tuning, n, dtype, m);
    const TuningResolved &tm = ms.tm;
    const bool reg = ms.reg, anchor = ms.anchor;
    // H psi (the adjoint's lam) on the same kernel family: psi and lam in
    // registers, both moved through half-tile LDS buffers, so the tile is at
    // most 2^13 (at 2^14 the 1,024-thread workgroups cannot hold psi and lam
    // of 16 amplitudes each without spilling), with at least 256 tiles
    TuningResolved th = tm;
    th.tile_bits = std::min(tm.tile_bits, 13);
    th.tile_bits = std::min(th.tile_bits, std::max(n - 8, std::min(n, 10)));
    if (th.tile_bits < n) th.low_bits = std::min(th.low_bits, th.tile_bits - 1);
    std::vector<Pauli> tp(reg ? m : 0);
    for (size_t i = 0; i < tp.size(); ++i) tp[i] = Pauli{terms[i].x, terms[i].z, terms[i].e & 3};
    PlanJob jm([&] { return term_passes(n, dtype, groups, tp, tm, anchor, h->margs, "cfh_ham_create"); });
    PlanJob jh([&] { return term_passes(n, dtype, groups, tp, th, true, h->hargs, "cfh_ham_create"); });
    if (reg) {
        jm.start();
        jh.start();
    }
    h->passes = plan_hamiltonian(n, groups, h->tu);
    std::vector<HamGroupDev> gdev;
    std::vector<HamTermDev> tdev;
    for (const HamPass &hp : h->passes) {
        HamPassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.outer_mask = hp.outer_mask;
        for (int j = 0; j < hp.b; ++j) a.v[j] = hp.v[j];
        a.b = hp.b;
        a.group_begin = (int32_t)gdev.size();
        a.group_count = (int32_t)hp.groups.size();
        for (int g : hp.groups) {
            bool in_span = false;
            HamGroupDev gd;
            gd.xl = local_coords(hp.v, groups[g].x, &in_span);
            if (!in_span) return set_error(CFH_E_INVAL, "Hamiltonian planner produced a group outside its tile");
            gd.hb = gd.xl ? 31 - __builtin_clz(gd.xl) : -1;
            gd.term_begin = (int32_t)tdev.size();
            gd.term_count = (int32_t)groups[g].terms.size();
            for (int i : groups[g].terms) {
                HamTermDev td;
                td.z = terms[i].z;
                td.zl = local_zmask(hp.v, terms[i].z);
                td.pad = 0;
                const int wp = (terms[i].e - popc(terms[i].x & terms[i].z)) & 3;  // i^wp
                const double c = coeff[i];
                td.wre = (wp == 0) ? c : (wp == 2) ? -c : 0.0;
                td.wim = (wp == 1) ? c : (wp == 3) ? -c : 0.0;
                tdev.push_back(td);
            }
            gdev.push_back(gd);
        }
        h->args.push_back(a);
    }
    cfh_status st = CFH_OK;
    std::vector<double2> mw_host;  // weights of the register-tiled passes' terms
    if (reg) {
        if ((st = jm.finish()) || (st = jh.finish())) return st;
        mw_host.resize(m);
        for (size_t i = 0; i < m; ++i) {
            const int wp = (terms[i].e - popc(terms[i].x & terms[i].z)) & 3;  // i^wp
            mw_host[i] = make_double2(wp == 0 ? coeff[i] : wp == 2 ? -coeff[i] : 0.0,
                                      wp == 1 ? coeff[i] : wp == 3 ? -coeff[i] : 0.0);
        }
        h->mmode = anchor ? 14 : 10;
    }
    // Device calls come only after all host planning: hipMemcpy on the null
    // stream waits for work already queued there, and planning done after it
    // would leave the device idle.
    if (!gdev.empty()) {
        if (!hip_ok(hipMalloc(&h->groups, gdev.size() * sizeof(HamGroupDev)), "cfh_ham_create: hipMalloc", &st) ||
            !hip_ok(hipMemcpy(h->groups, gdev.data(), gdev.size() * sizeof(HamGroupDev), hipMemcpyHostToDevice),
                    "cfh_ham_create: hipMemcpy", &st) ||
            !hip_ok(hipMalloc(&h->terms, tdev.size() * sizeof(HamTermDev)), "cfh_ham_create: hipMalloc", &st) ||
            !hip_ok(hipMemcpy(h->terms, tdev.data(), tdev.size() * sizeof(HamTermDev), hipMemcpyHostToDevice),
                    "cfh_ham_create: hipMemcpy", &st))
            return st;
    }
    if (!mw_host.empty() &&
        (!hip_ok(hipMalloc(&h->mw, m * sizeof(double2)), "cfh_ham_create: hipMalloc", &st) ||
         !hip_ok(hipMemcpy(h->mw, mw_host.data(), m * sizeof(double2), hipMemcpyHostToDevice),
                 "cfh_ham_create: hipMemcpy", &st)))
        return st;
    h->grid = persistent_grid(1ull << (n - h->tu.tile_bits));
    const size_t np = std::max<size_t>(h->grid, cfh_ham_s::kMeasureGrid);
    if (!hip_ok(hipMalloc(&h->partial, np * sizeof(double2)), "cfh_ham_create: hipMalloc", &st)) return st;
    *out = h.release();
    return CFH_OK;
}

cfh_status cfh_ham_destroy(cfh_ham h)
{
    delete h;
    return CFH_OK;
}

cfh_status cfh_ham_info(cfh_ham h, int64_t *n_passes, int64_t *n_groups, double *hbm_bytes)
{
    if (!h) return set_error(CFH_E_INVAL, "cfh_ham_info: null");
    const size_t np = h->mmode ? h->margs.size() : h->args.size();  // read passes of one <H>
    if (n_passes) *n_passes = (int64_t)np;
    if (n_groups) *n_groups = h->n_groups;
    if (hbm_bytes) *hbm_bytes = (double)np * (double)(1ull << h->n) * (double)amp_bytes(h->dtype);
    return CFH_OK;
}

cfh_status cfh_expval_async(cfh_ham h, const void *psi, double *out_dev, void *stream)
{
    if (!h || !psi || !out_dev) return set_error(CFH_E_INVAL, "cfh_expval_async: null argument");
    hipStream_t s = (hipStream_t)stream;
    if (h->mmode) {
        const unsigned G = cfh_ham_s::kMeasureGrid;
        hipLaunchKernelGGL(k_zero_d, dim3((2 * G + 255) / 256), dim3(256), 0, s, (double *)h->partial,
                           (int64_t)(2 * G));
        cfh_status st = last_launch("k_zero_d");
        if (st) return st;
        for (const PassArgs2 &a : h->margs) {
            const uint64_t ntiles = 1ull << (h->n - a.b);
            st = h->dtype == CFH_C128
                     ? launch_pass2(ntiles, s, (double2 *)const_cast<void *>(psi), h->mw, a, h->mmode, h->partial, G)
                     : launch_pass2(ntiles, s, (float2 *)const_cast<void *>(psi), h->mw, a, h->mmode, h->partial, G);
            if (st) return st;
        }
        hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, s, h->partial, (int)G, out_dev);
        return last_launch("k_reduce_partial");
    }
    const int cnt = (int)h->grid * 2;
    hipLaunchKernelGGL(k_zero_d, dim3((cnt + 255) / 256), dim3(256), 0, s, (double *)h->partial, (int64_t)cnt);
    cfh_status st = last_launch("k_zero_d");
    if (st) return st;
    for (const HamPassArgs &a : h->args) {
        const uint64_t ntiles = 1ull << (h->n - a.b);
        st = h->dtype == CFH_C128
                 ? launch_ham(a.b, ntiles, h->grid, s, (const double2 *)psi, (double2 *)nullptr, a, h->groups,
                              h->terms, h->partial, 0)
                 : launch_ham(a.b, ntiles, h->grid, s, (const float2 *)psi, (float2 *)nullptr, a, h->groups,
                              h->terms, h->partial, 0);
        if (st) return st;
    }
    hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, s, h->partial, (int)h->grid, out_dev);
    return last_launch("k_reduce_partial");
}

cfh_status cfh_ham_apply(cfh_ham h, const void *psi, void *out, void *stream)
{
    if (!h || !psi || !out) return set_error(CFH_E_INVAL, "cfh_ham_apply: null argument");
    if (psi == out) return set_error(CFH_E_INVAL, "cfh_ham_apply: out must not alias psi");
    hipStream_t s = (hipStream_t)stream;
    if (h->args.empty()) {
        const uint64_t cnt = (1ull << h->n) * amp_bytes(h->dtype) / 8;
        hipLaunchKernelGGL(k_zero_d, dim3((unsigned)std::min<uint64_t>((cnt + 255) / 256, 1u << 20)), dim3(256), 0, s,
                           (double *)out, (int64_t)cnt);
        return last_launch("k_zero_d");
    }
    if (!h->hargs.empty()) {
        for (size_t i = 0; i < h->hargs.size(); ++i) {
            const PassArgs2 &a = h->hargs[i];
            const uint64_t ntiles = 1ull << (h->n - a.b);
            cfh_status st = h->dtype == CFH_C128
                                ? launch_ham2(ntiles, s, (const double2 *)psi, (double2 *)out, h->mw, a, i > 0)
                                : launch_ham2(ntiles, s, (const float2 *)psi, (float2 *)out, h->mw, a, i > 0);
            if (st) return st;
        }
        return CFH_OK;
    }
    for (size_t i = 0; i < h->args.size(); ++i) {
        const HamPassArgs &a = h->args[i];
        const uint64_t ntiles = 1ull << (h->n - a.b);
        cfh_status st = h->dtype == CFH_C128
                            ? launch_ham(a.b, ntiles, 0, s, (const double2 *)psi, (double2 *)out, a, h->groups,
                                         h->terms, nullptr, i > 0)
                            : launch_ham(a.b, ntiles, 0, s, (const float2 *)psi, (float2 *)out, a, h->groups,
                                         h->terms, nullptr, i > 0);
        if (st) return st;
    }
    return CFH_OK;
}

cfh_status cfh_expval(const void *psi, int n, int dtype, const cfh_pauli *terms, const double *coeff, size_t m,
                      double *out_host, void *stream)
{
    if (!out_host) return set_error(CFH_E_INVAL, "cfh_expval: null output");
    cfh_status st = check_state_args(psi, n, dtype, "cfh_expval");
    if (st) return st;
    cfh_ham h = nullptr;
    st = cfh_ham_create(n, dtype, terms, coeff, m, nullptr, &h);
    if (st) return st;
    double *d = nullptr;
    if (!hip_ok(hipMalloc(&d, 2 * sizeof(double)), "cfh_expval: hipMalloc", &st)) {
        cfh_ham_destroy(h);
        return st;
    }
    st = cfh_expval_async(h, psi, d, stream);
    if (!st && hip_ok(hipStreamSynchronize((hipStream_t)stream), "cfh_expval: sync", &st))
        hip_ok(hipMemcpy(out_host, d, 2 * sizeof(double), hipMemcpyDeviceToHost), "cfh_expval: copy", &st);
    (void)hipFree(d);
    cfh_ham_destroy(h);
    return st;
}

// ------------------------------------------------------------- adjoint
cfh_status cfh_adjoint_grad(cfh_plan p, cfh_ham h, void *psi, void *lam, const double *theta_dev, double *grad_dev,
                            void *stream)
{
    if (!p || !h || !psi || !lam || !grad_dev || (!theta_dev && !p->rot.empty()))
        return set_error(CFH_E_INVAL, "cfh_adjoint_grad: null argument");
    if (p->n != h->n || p->dtype != h->dtype)
        return set_error(CFH_E_INVAL, "cfh_adjoint_grad: plan and Hamiltonian differ in n or dtype");
    hipStream_t s = (hipStream_t)stream;
    cfh_status st = cfh_ham_apply(h, psi, lam, stream);
    if (st) return st;
    const int64_t m = (int64_t)p->rot.size();
    if (m == 0) return CFH_OK;
    hipLaunchKernelGGL(k_coef, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, theta_dev, p->coef, m);
    if ((st = last_launch("k_coef"))) return st;
    if (!p->adj2_args.empty()) {
        for (int64_t i = (int64_t)p->adj2_args.size() - 1; i >= 0; --i) {
            const PassArgs2 &a = p->adj2_args[i];
            const uint64_t ntiles = 1ull << (p->n - a.b);
            st = p->dtype == CFH_C128
                     ? launch_adj2(ntiles, s, (double2 *)psi, (double2 *)lam, p->coef, a, true, p->gpart,
                                   cfh_plan_s::kAdj2Grid, grad_dev)
                     : launch_adj2(ntiles, s, (float2 *)psi, (float2 *)lam, p->coef, a, true, p->gpart,
                                   cfh_plan_s::kAdj2Grid, grad_dev);
            if (st) return st;
        }
        return CFH_OK;
    }
    for (int64_t i = (int64_t)p->adj_args.size() - 1; i >= 0; --i) {
        const PassArgs &a = p->adj_args[i];
        const uint64_t ntiles = 1ull << (p->n - a.b);
        const unsigned grid = (unsigned)std::min<uint64_t>(ntiles, p->adj_grid);
        st = p->dtype == CFH_C128
                 ? launch_adjoint(a.b, ntiles, grid, s, (double2 *)psi, (double2 *)lam, p->coef, a, p->gpart)
                 : launch_adjoint(a.b, ntiles, grid, s, (float2 *)psi, (float2 *)lam, p->coef, a, p->gpart);
        if (st) return st;
        hipLaunchKernelGGL(k_grad_reduce, dim3(a.nrot), dim3(256), 0, s, p->gpart, (int)grid, a, grad_dev);
        if ((st = last_launch("k_grad_reduce"))) return st;
    }
    return CFH_OK;
}

// ------------------------------------------------------- device frame map
cfh_status cfh_frame_conjugate_device(cfh_frame f, const cfh_pauli *in_dev, cfh_pauli *out_dev, size_t m,
                                      void *stream)
{
    if (!f || (m && (!in_dev || !out_dev))) return set_error(CFH_E_INVAL, "cfh_frame_conjugate_device: null");
    if (m == 0) return CFH_OK;
    std::vector<FrameRowDev> rows(2 * f->n);
    for (int q = 0; q < f->n; ++q) {
        rows[q] = FrameRowDev{f->zf[q].x, f->zf[q].z, f->zf[q].e, 0};
        rows[f->n + q] = FrameRowDev{f->xf[q].x, f->xf[q].z, f->xf[q].e, 0};
    }
    FrameRowDev *d = nullptr;
    cfh_status st = CFH_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!hip_ok(hipMalloc((void **)&d, rows.size() * sizeof(FrameRowDev)), "hipMalloc", &st)) return st;
    if (!hip_ok(hipMemcpy(d, rows.data(), rows.size() * sizeof(FrameRowDev), hipMemcpyHostToDevice), "hipMemcpy",
                &st)) {
        (void)hipFree(d);
        return st;
    }
    hipLaunchKernelGGL(k_frame_conjugate, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, d, f->n, in_dev,
                       out_dev, (uint64_t)m);
    st = last_launch("k_frame_conjugate");
    // the row copy is freed only after the kernel that reads it has finished
    cfh_status st2 = CFH_OK;
    hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st2);
    (void)hipFree(d);
    return st ? st : st2;
}

} // extern "C"

namespace {

// Plan the rotations, apply them to psi on `stream` and wait (the angle buffer
// and the plan are freed before returning).
cfh_status run_rotations(int n, int dtype, const std::vector<cfh_pauli> &rot, const std::vector<double> &th,
                         const cfh_tuning *tuning, void *psi, void *stream, const char *what)
{
    if (rot.empty()) return CFH_OK;
    cfh_plan p = nullptr;
    cfh_status st = cfh_plan_create(n, dtype, rot.data(), rot.size(), tuning, &p);
    if (st) return st;
    double *d = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (hip_ok(hipMalloc(&d, th.size() * sizeof(double)), what, &st) &&
        hip_ok(hipMemcpyAsync(d, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice, s), what, &st)) {
        st = cfh_apply_plan(p, psi, d, 0, stream);
        cfh_status st2 = CFH_OK;
        hip_ok(hipStreamSynchronize(s), what, &st2);
        if (!st) st = st2;
    }
    if (d) (void)hipFree(d);
    cfh_plan_destroy(p);
    return st;
}

} // namespace

extern "C" {

cfh_status cfh_frame_flush(cfh_frame f, void *psi, int dtype, void *stream)
{
    if (!f || !psi) return set_error(CFH_E_INVAL, "cfh_frame_flush: null argument");
    std::vector<Pauli> q;
    std::vector<double> th;
    cfh_status st = frame_flush_rotations(*f, q, th);
    if (st) return st;
    std::vector<cfh_pauli> rot(q.size());
    for (size_t i = 0; i < q.size(); ++i) rot[i] = cfh_pauli{q[i].x, q[i].z, q[i].e, 0};
    st = run_rotations(f->n, dtype, rot, th, nullptr, psi, stream, "cfh_frame_flush");
    if (st) return st;
    frame_reset(*f);
    return CFH_OK;
}

cfh_status cfh_circuit_run(cfh_frame f, const int32_t *gates, const double *angles, size_t m, void *psi, int dtype,
                           const cfh_tuning *tuning, int32_t *outcomes, void *stream)
{
    if (!f || !psi || (m && !gates)) return set_error(CFH_E_INVAL, "cfh_circuit_run: null argument");
    std::vector<cfh_pauli> rot;
    std::vector<double> th;
    size_t i = 0;
    while (true) {
        // the rows up to the next measurement or reset: frame updates and rotations
        size_t stop = 0;
        cfh_status st = circuit_translate(*f, gates, angles, i, m, rot, th, &stop);
        if (st) return st;
        st = run_rotations(f->n, dtype, rot, th, tuning, psi, stream, "cfh_circuit_run");
        if (st) return st;
        if (stop >= m) return CFH_OK;
        const int code = gates[3 * stop], q = gates[3 * stop + 1];
        if (q < 0 || q >= f->n || gates[3 * stop + 2] != -1 || !angles || !outcomes)
            return set_error(CFH_E_INVAL, "cfh_circuit_run: a measurement or reset needs q0 in range, q1 = -1, "
                                          "its uniform number in angles and an outcomes array");
        // measuring Z_q on U Phi is measuring F(Z_q) on Phi (the frame axis)
        cfh_pauli zq{0, 1ull << q, 0, 0}, pz{}, px{};
        st = cfh_frame_conjugate(f, &zq, &pz);
        if (st) return st;
        int32_t out = 0;
        st = cfh_measure_pauli(psi, f->n, dtype, &pz, angles[stop], &out, nullptr, stream);
        if (st) return st;
        outcomes[stop] = out;
        if (code == CFH_GATE_RESET && out < 0) {
            // X_q on U Phi is F(X_q) on Phi; exp(-i pi/2 Q) = -i Q applies it up to a global phase
            cfh_pauli xq{1ull << q, 0, 0, 0};
            st = cfh_frame_conjugate(f, &xq, &px);
            if (st) return st;
            st = cfh_apply_pauli_rotation(psi, f->n, dtype, px.x, px.z, px.e, 3.14159265358979323846, stream);
            if (st) return st;
        }
        i = stop + 1;
    }
}

} // extern "C"
