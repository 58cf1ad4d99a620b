// Register-tiled fused pass kernel (k_pass2) and its launcher.  Included by
// one translation unit per storage type so the two instantiations compile in
// parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>

#include "cfh_internal.hpp"
#include "device_common.hpp"
#include "launch.hpp"

namespace {

using namespace cfh;
using namespace cfh::dev;

// ------------------------------------------ register-tiled fused pass (v2)
// Thread t of a workgroup holds, during micro-group g, the 16 amplitudes
// a = base_t ^ U_g[j] of the coset, base_t = deposit(t, npiv_g).  A rotation
// of the micro-group pairs registers j and j ^ cx (cx known only at run time
// but uniform, so it selects one of 15 unrolled bodies).  Member j of the
// pair gets the sign (-1)^{parity(y & z)} = (-1)^{st ^ msign_j}, with st the
// thread/coset part and msign_j the register part precomputed on the host.
// Workgroups are persistent: the loads of the next coset are issued before
// the current one is processed, so HBM traffic overlaps the arithmetic.

__device__ __forceinline__ uint32_t deposit32(uint32_t v, uint32_t mask)
{
    uint32_t r = 0;
    for (uint32_t m = mask; m && v; m &= m - 1, v >>= 1)
        if (v & 1) r |= m & (~m + 1);
    return r;
}

// deposit32(t, mask) for the thread index t of a workgroup of at least one
// wave, where mask has one set bit per thread-index bit: the six lane bits go
// to the six lowest set bits of mask (two VALU operations each), the wave
// bits, uniform across the wave, to the others (scalar operations).
__device__ __forceinline__ uint32_t deposit_tid(uint32_t t, uint32_t mask)
{
    uint32_t m = mask, r = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const uint32_t low = m & (~m + 1);
        r |= (0u - ((t >> i) & 1u)) & low;
        m &= m - 1;
    }
    return r | deposit32(__builtin_amdgcn_readfirstlane(t >> 6), m);
}

// v with its sign flipped when the (wave-uniform) bit is set: one XOR of the
// high word instead of a select between two registers.
__device__ __forceinline__ double flip_if(double v, uint32_t bit)
{
    return __longlong_as_double(__double_as_longlong(v) ^ ((unsigned long long)(bit & 1) << 63));
}

template <int CX, bool IMAG>
__device__ __forceinline__ void mg_rot(double2 (&r)[kRegs], double c, double srA, uint32_t msign)
{
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
        if ((j ^ CX) > j) {
            const double s0 = flip_if(srA, msign >> j);
            const double s1 = flip_if(srA, msign >> (j ^ CX));
            rot_pair(r[j], r[j ^ CX], c, s0, s1, IMAG);
            // pairs one after another: the scheduler would otherwise keep the
            // temporaries of all eight pairs live at once
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <bool IMAG>
__device__ __forceinline__ void mg_diag(double2 (&r)[kRegs], double c, double srA, uint32_t msign)
{
#pragma unroll
    for (int j = 0; j < kRegs; ++j) r[j] = rot_diag(r[j], c, flip_if(srA, msign >> j), IMAG);
}


template <bool IMAG>
__device__ __forceinline__ void mg_dispatch(int cx, double2 (&r)[kRegs], double c, double srA, uint32_t msign)
{
    switch (cx) {
    case 0: mg_diag<IMAG>(r, c, srA, msign); break;
    case 1: mg_rot<1, IMAG>(r, c, srA, msign); break;
    case 2: mg_rot<2, IMAG>(r, c, srA, msign); break;
    case 3: mg_rot<3, IMAG>(r, c, srA, msign); break;
    case 4: mg_rot<4, IMAG>(r, c, srA, msign); break;
    case 5: mg_rot<5, IMAG>(r, c, srA, msign); break;
    case 6: mg_rot<6, IMAG>(r, c, srA, msign); break;
    case 7: mg_rot<7, IMAG>(r, c, srA, msign); break;
    case 8: mg_rot<8, IMAG>(r, c, srA, msign); break;
    case 9: mg_rot<9, IMAG>(r, c, srA, msign); break;
    case 10: mg_rot<10, IMAG>(r, c, srA, msign); break;
    case 11: mg_rot<11, IMAG>(r, c, srA, msign); break;
    case 12: mg_rot<12, IMAG>(r, c, srA, msign); break;
    case 13: mg_rot<13, IMAG>(r, c, srA, msign); break;
    case 14: mg_rot<14, IMAG>(r, c, srA, msign); break;
    default: mg_rot<15, IMAG>(r, c, srA, msign); break;
    }
}

// Compile-time rotation bodies.  KASE = cx | zr << 4 fixes the partner mask
// and every register's sign (the sign of register j is parity(j & zr), since
// the register offsets are spanned by four vectors), so the signs become
// negations of FMA operands instead of sign arithmetic.  For a Hermitian
// rotation the pair coefficient is imaginary exactly when |x & z| is even,
// and |x & z| = parity(cx & zr) in register coordinates, so KASE also fixes
// real/imaginary: 256 bodies cover every rotation the planner emits (the
// planner checks the relation for each descriptor).
constexpr bool cpar(int v) { return __builtin_popcount(v) & 1; }

// TAN: the tangent form of the same update, c(u + t sigma beta v) with
// t = s / c: the factor c is left out (the caller applies the product of the
// pass's factors at the end), so a pair costs 4 FMAs instead of 4 MULs and
// 4 FMAs.  Callers pass c = 1 and s = t.
template <int KASE, bool TAN = false>
__device__ __forceinline__ void kase_body(double2 (&r)[kRegs], double c_in, double s)
{
    const double c = TAN ? 1.0 : c_in;
    constexpr int CX = KASE & 15, ZR = (KASE >> 4) & 15;
    constexpr bool IMAG = CX == 0 || !cpar(CX & ZR);
    if constexpr (CX == 0) {
        // x = 0: exp(-i theta/2 P) is a phase on every amplitude
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            const double sj = cpar(j & ZR) ? -s : s;
            r[j] = make_double2(c * r[j].x - sj * r[j].y, c * r[j].y + sj * r[j].x);
        }
    } else {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if ((j ^ CX) > j) {
                rot_pair(r[j], r[j ^ CX], c, cpar(j & ZR) ? -s : s, cpar((j ^ CX) & ZR) ? -s : s, IMAG);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// One leaf per body, selected by a dense switch on cx | zr << 4 (a binary
// search of scalar compares, two scalar instructions per level).
#define CFH_KASE_CASE(K) \
    case K: kase_body<K, TAN>(r, c, s); break;
#define CFH_KASE_CASE4(K) CFH_KASE_CASE(K) CFH_KASE_CASE(K + 1) CFH_KASE_CASE(K + 2) CFH_KASE_CASE(K + 3)
#define CFH_KASE_CASE16(K) CFH_KASE_CASE4(K) CFH_KASE_CASE4(K + 4) CFH_KASE_CASE4(K + 8) CFH_KASE_CASE4(K + 12)
#define CFH_KASE_CASE64(K) CFH_KASE_CASE16(K) CFH_KASE_CASE16(K + 16) CFH_KASE_CASE16(K + 32) CFH_KASE_CASE16(K + 48)
template <bool TAN = false>
__device__ __forceinline__ void kase_switch(uint32_t kase, double2 (&r)[kRegs], double c, double s)
{
    switch (kase & 255u) {
        CFH_KASE_CASE64(0) CFH_KASE_CASE64(64) CFH_KASE_CASE64(128) CFH_KASE_CASE64(192)
    default: break;
    }
}
#undef CFH_KASE_CASE64
#undef CFH_KASE_CASE16
#undef CFH_KASE_CASE4
#undef CFH_KASE_CASE

// Read-only term bodies (expectation values).  For a term with partner mask
// CX and register sign mask ZR (the sign of register j is
// sigma_j = (-1)^{parity(j & ZR)}, as for the rotation bodies) the thread's
// share of
//   sum_y (-1)^{|y & z|} conj(psi_y) psi_{y ^ x}
// is (thread and coset sign) * S, S = sum_j sigma_j conj(r_j) r_{j^CX}.  The
// members j and j^CX of a pair give conjugate products, and
// sigma_{j^CX} = sigma_j sigma_CX, so S = 2 sum_{j<j^CX} sigma_j Re(conj(r_j) r_{j^CX})
// when sigma_CX = +1 and 2i sum sigma_j Im(...) when sigma_CX = -1; for
// CX = 0, S = sum_j sigma_j |r_j|^2.  With ZR fixed at compile time every sign
// is an FMA operand negation: a pair costs two FMAs, accumulated into two
// independent partial sums.
template <int KM>
__device__ __forceinline__ void meas_body(const double2 (&r)[kRegs], double wre, double wim, double &accr,
                                          double &acci)
{
    constexpr int CX = KM & 15, ZR = (KM >> 4) & 15;
    double acc[2] = {0.0, 0.0};
    if constexpr (CX == 0) {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            const double x = cpar(j & ZR) ? -r[j].x : r[j].x;
            const double y = cpar(j & ZR) ? -r[j].y : r[j].y;
            acc[j & 1] = fma(x, r[j].x, acc[j & 1]);
            acc[j & 1] = fma(y, r[j].y, acc[j & 1]);
        }
        const double S = acc[0] + acc[1];
        accr = fma(wre, S, accr);
        acci = fma(wim, S, acci);
    } else {
        constexpr bool IM = cpar(CX & ZR);
        constexpr int LOW = CX & -CX;           // j runs over the pair members with this bit clear
        constexpr int ALT = LOW == 1 ? 2 : 1;   // alternates over those members: two partial sums
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if (j & LOW) continue;
            const double2 a = r[j], b = r[j ^ CX];
            const bool neg = cpar(j & ZR);
            double &t = acc[(j & ALT) ? 1 : 0];
            if constexpr (IM) {
                t = fma(neg ? -a.x : a.x, b.y, t);
                t = fma(neg ? a.y : -a.y, b.x, t);
            } else {
                t = fma(neg ? -a.x : a.x, b.x, t);
                t = fma(neg ? -a.y : a.y, b.y, t);
            }
        }
        const double S = 2.0 * (acc[0] + acc[1]);
        if constexpr (IM) {
            accr = fma(-wim, S, accr);
            acci = fma(wre, S, acci);
        } else {
            accr = fma(wre, S, accr);
            acci = fma(wim, S, acci);
        }
    }
}

// One leaf per body, selected by a dense switch on cx | zr << 4.
#define CFH_MEAS_CASE(K) \
    case K: meas_body<K>(r, wre, wim, accr, acci); break;
#define CFH_MEAS_CASE4(K) CFH_MEAS_CASE(K) CFH_MEAS_CASE(K + 1) CFH_MEAS_CASE(K + 2) CFH_MEAS_CASE(K + 3)
#define CFH_MEAS_CASE16(K) CFH_MEAS_CASE4(K) CFH_MEAS_CASE4(K + 4) CFH_MEAS_CASE4(K + 8) CFH_MEAS_CASE4(K + 12)
#define CFH_MEAS_CASE64(K) CFH_MEAS_CASE16(K) CFH_MEAS_CASE16(K + 16) CFH_MEAS_CASE16(K + 32) CFH_MEAS_CASE16(K + 48)
__device__ __forceinline__ void meas_switch(uint32_t km, const double2 (&r)[kRegs], double wre, double wim,
                                            double &accr, double &acci)
{
    switch (km & 255u) {
        CFH_MEAS_CASE64(0) CFH_MEAS_CASE64(64) CFH_MEAS_CASE64(128) CFH_MEAS_CASE64(192)
    default: break;
    }
}
#undef CFH_MEAS_CASE64
#undef CFH_MEAS_CASE16
#undef CFH_MEAS_CASE4
#undef CFH_MEAS_CASE

// Coset handled at loop index t of the persistent loop.  Workgroups are
// dealt to the 8 XCDs in turn (workgroup w runs on XCD w mod 8) and the grid
// is a multiple of 8 when p > 0, so loop indices t and t + 8j (j < 2^p) run on
// one XCD at the same time.  The 2^p cosets whose amplitudes share 128-byte
// lines differ only in their low p index bits; they get loop indices 8 apart,
// so each line is filled into that XCD's L2 once and written back whole.
// Needs 8 * 2^p <= ntiles (both powers of two): then this is a permutation.
__device__ __forceinline__ uint64_t coset_of(uint64_t t, int p, uint64_t ntiles)
{
    if (p == 0) return t;
    if (p < 0) {
        // bit-reversed order: workgroups running at the same time are spread
        // over the whole state (ntiles is a power of two)
        const int lg = 63 - __builtin_clzll(ntiles);
        return lg == 0 ? t : (__brevll(t) >> (64 - lg));
    }
    const uint64_t m = (8ull << p) - 1, lo = t & m;
    return (t & ~m) | ((lo & 7) << p) | (lo >> 3);
}

// MODE bit 0: prefetch the next coset into registers.
// MODE bit 1: compile-time rotation bodies; (c, s) of the pass staged in LDS
//             once per workgroup, thread signs precomputed as one bit mask.
// MODE bit 2: half-tile transposes.  Register dimension 0 of every
//             micro-group is the same anchor vector, whose pivot is local
//             bit qbit; so the amplitudes with local bit qbit = h are exactly
//             the registers j with (j & 1) == h in both layouts, and each half
//             moves through an LDS buffer of 2^(B-1) amplitudes indexed by the
//             local coordinate with bit qbit removed.
// MODE bit 3: read-only measurement (with bit 1): the descriptors are terms
//             of an observable, coef holds their weights w_k = c_k i^{(e-|x&z|)},
//             nothing is stored and each workgroup adds its share of
//             sum_k w_k <psi|P_k|psi> to partial[blockIdx.x].
template <typename Amp, int B, int MODE>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_pass2(Amp *__restrict__ psi, const double2 *__restrict__ coef, const PassArgs2 args, uint64_t ntiles,
        double2 *__restrict__ partial)
{
    constexpr bool PF = MODE & 1;
    constexpr bool CT = MODE & 2;
    constexpr bool HALF = MODE & 4;
    constexpr bool MEAS = MODE & 8;
    constexpr bool TANF = MODE & 16;
    static_assert(!MEAS || (CT && !PF), "measurement uses the compile-time bodies without prefetch");
    static_assert(!TANF || (CT && !MEAS), "the tangent form needs the compile-time rotation bodies");
    constexpr int NW = (1 << (B - kRegDims)) / 64;  // waves per workgroup
    extern __shared__ unsigned char lds_raw[];
    Amp *lds = reinterpret_cast<Amp *>(lds_raw);
    __shared__ double2 tab[CT ? kMaxRun : 1];
    __shared__ double2 red[MEAS ? NW : 1];
    const uint32_t t = threadIdx.x;
    const int last = args.nmg - 1;
    uint32_t tsb = 0;  // bit ri: parity(t & zt) of rotation ri
    uint32_t tanm = 0; // bit ri: rotation ri runs in the tangent form (|s| <= |c|)
    double gscale = 1.0;  // product of c over the tangent-form rotations
    double accr = 0.0, acci = 0.0;
    if constexpr (CT) {
        const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
        if ((int)t < nrot) {
            const RotDesc2 &d = args.rot[t];
            const double2 cs = coef[d.k];
            if constexpr (MEAS) {
                tab[t] = cs;
            } else {
                double sv = args.inverse ? -cs.y : cs.y;
                if (d.flags & 2) sv = -sv;
                tab[t] = make_double2(cs.x, sv);
            }
        }
        for (int ri = 0; ri < nrot; ++ri) tsb |= (uint32_t)par32(t & args.rot[ri].zt) << ri;
        __syncthreads();
        if constexpr (TANF) {
            // every thread forms the same mask and product, in the same order
            for (int ri = 0; ri < nrot; ++ri) {
                const double2 cs = tab[ri];
                if (fabs(cs.y) <= fabs(cs.x)) {
                    tanm |= 1u << ri;
                    gscale *= cs.x;
                }
            }
            __syncthreads();
            if ((int)t < nrot && ((tanm >> t) & 1)) tab[t].y = tab[t].y / tab[t].x;
            __syncthreads();
        }
    }
    uint64_t Lb0 = 0, LbL = 0;
    {
        const uint32_t b0 = deposit32(t, args.mg[0].npiv), bL = deposit32(t, args.mg[last].npiv);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if ((b0 >> i) & 1) Lb0 ^= args.v[i];
            if ((bL >> i) & 1) LbL ^= args.v[i];
        }
    }
    Amp pf[kRegs];
    uint64_t tile = blockIdx.x;
    if (PF && tile < ntiles) {
        const uint64_t y0 = deposit(coset_of(tile, args.xrot, ntiles), args.outer_mask) ^ Lb0;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) pf[j] = psi[y0 ^ args.LU_first[j]];
    }
#pragma unroll 1
    for (; tile < ntiles; tile += gridDim.x) {
        // keep the 2 x 16 per-register address terms from being hoisted out of
        // the loop as 64 live VGPRs: recomputing them is two scalar-operand XORs
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(coset_of(tile, args.xrot, ntiles), args.outer_mask);
        double2 r[kRegs];
        if (PF) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) r[j] = ld(pf[j]);
            const uint64_t nt = tile + gridDim.x;
            if (nt < ntiles) {
                const uint64_t y0 = deposit(coset_of(nt, args.xrot, ntiles), args.outer_mask) ^ Lb0;
#pragma unroll
                for (int j = 0; j < kRegs; ++j) pf[j] = psi[y0 ^ args.LU_first[j]];
            }
        } else {
            const uint64_t y0 = tb ^ Lb0;
#pragma unroll
            for (int j = 0; j < kRegs; ++j) r[j] = ld(psi[y0 ^ args.LU_first[j]]);
        }
        uint32_t bprev = 0;
#pragma unroll 1
        for (int g = 0; g <= last; ++g) {
            const MGDesc2 &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const MGDesc2 &mp = args.mg[g - 1];
                if constexpr (HALF) {
                    // bprev and bt have 0 at the anchor bit (it is a pivot)
                    const uint32_t lo = (1u << args.qbit) - 1;
                    const uint32_t bw = (bprev & lo) | ((bprev >> 1) & ~lo);
                    const uint32_t br = (bt & lo) | ((bt >> 1) & ~lo);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
#pragma unroll
                        for (int j = h; j < kRegs; j += 2) st(lds[bw ^ mp.UC[j]], r[j]);
                        __syncthreads();
#pragma unroll
                        for (int j = h; j < kRegs; j += 2) r[j] = ld(lds[br ^ m.UC[j]]);
                        __syncthreads();
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) st(lds[bprev ^ mp.U[j]], r[j]);
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) r[j] = ld(lds[bt ^ m.U[j]]);
                    __syncthreads();
                }
            }
            bprev = bt;
            if constexpr (MEAS) {
#pragma unroll 1
                for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                    // the amplitudes do not change between terms: without this the
                    // products of all 15 partner masks get hoisted out of the loop
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) asm volatile("" : "+v"(r[j].x), "+v"(r[j].y));
                    const RotDesc2 &d = args.rot[ri];
                    const double2 w = tab[ri];
                    const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                    meas_switch(d.kase, r, flip_if(w.x, sg), flip_if(w.y, sg), accr, acci);
                }
            } else if constexpr (CT) {
#pragma unroll 1
                for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                    const RotDesc2 &d = args.rot[ri];
                    const double2 cs = tab[ri];
                    const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                    if (TANF && ((tanm >> ri) & 1))
                        kase_switch<true>(d.kase, r, 1.0, flip_if(cs.y, sg));
                    else
                        kase_switch(d.kase, r, cs.x, flip_if(cs.y, sg));
                }
            } else {
#pragma unroll 1
                for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                    const RotDesc2 &d = args.rot[ri];
                    const double2 cs = coef[d.k];
                    double sr = args.inverse ? -cs.y : cs.y;
                    if (d.flags & 2) sr = -sr;
                    const int sg = par32(bt & d.zl) ^ par64(tb & d.z);
                    const double srA = sg ? -sr : sr;
                    if (d.flags & 1)
                        mg_dispatch<true>(d.cx, r, cs.x, srA, d.msign);
                    else
                        mg_dispatch<false>(d.cx, r, cs.x, srA, d.msign);
                }
            }
        }
        if constexpr (!MEAS) {
            if constexpr (TANF) {
#pragma unroll
                for (int j = 0; j < kRegs; ++j) r[j] = make_double2(r[j].x * gscale, r[j].y * gscale);
            }
            const uint64_t yL = tb ^ LbL;
#pragma unroll
            for (int j = 0; j < kRegs; ++j) st(psi[yL ^ args.LU_last[j]], r[j]);
        }
    }
    if constexpr (MEAS) {
        // fixed-order reduction: waves, then one add into this workgroup's slot
        accr = wave_sum<64>(accr);
        acci = wave_sum<64>(acci);
        if ((t & 63) == 0) red[t >> 6] = make_double2(accr, acci);
        __syncthreads();
        if (t == 0) {
            double sr = 0.0, si = 0.0;
            for (int i = 0; i < NW; ++i) {
                sr += red[i].x;
                si += red[i].y;
            }
            partial[blockIdx.x].x += sr;
            partial[blockIdx.x].y += si;
        }
    }
}

// ------------------------------------------------ register-tiled adjoint pass
// psi and lam of one coset in registers (16 amplitudes each per thread).  The
// run is walked backwards (inverse-order descriptors, angles negated): for
// each rotation the thread adds its share of Im <lam|P_k|psi> over the coset,
// then both vectors are rewound by R_k^dag with the same compile-time bodies
// as the forward pass.  With (P psi)_y = i^wp (-1)^{|y&z|} psi_{y^x} the share
// is (thread and coset sign) * Im(i^wp Z), Z = sum_j sigma_j conj(l_j) p_{j^cx}:
// Re Z for odd wp (real beta in the rotation), Im Z for even wp; the sign of
// i^wp is descriptor flag bit 2.  Per-wave sums accumulate in LDS over the
// cosets and are written per workgroup in a fixed order.
// The register signs are taken at run time from msign (bit j = sign of
// register j), so only the partner mask and real/imaginary beta select a body:
// 32 bodies of the two-vector update instead of 512.
template <int CX, bool IMAG>
__device__ __forceinline__ void adj_body(double2 (&p)[kRegs], double2 (&l)[kRegs], double c, double s,
                                         uint32_t msign, double &g)
{
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
        const double2 u = p[j ^ CX], v = l[j];
        g += flip_if(IMAG ? v.x * u.y - v.y * u.x : v.x * u.x + v.y * u.y, msign >> j);
    }
    if constexpr (CX == 0) {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            const double sj = flip_if(s, msign >> j);
            p[j] = rot_diag(p[j], c, sj, IMAG);
            l[j] = rot_diag(l[j], c, sj, IMAG);
        }
    } else {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if ((j ^ CX) > j) {
                const double s0 = flip_if(s, msign >> j), s1 = flip_if(s, msign >> (j ^ CX));
                rot_pair(p[j], p[j ^ CX], c, s0, s1, IMAG);
                rot_pair(l[j], l[j ^ CX], c, s0, s1, IMAG);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
}

// branch tree over bit 8 (imaginary beta) and bits 3..0 (partner mask) of kase
template <int BIT, int ACC>
__device__ __forceinline__ void adj_dispatch(uint32_t kase, double2 (&p)[kRegs], double2 (&l)[kRegs], double c,
                                             double s, uint32_t msign, double &g)
{
    if constexpr (BIT < 0) {
        adj_body<ACC & 15, (ACC >> 8) & 1>(p, l, c, s, msign, g);
    } else {
        constexpr int NEXT = BIT == 8 ? 3 : BIT - 1;
        if (kase & (1u << BIT))
            adj_dispatch<NEXT, ACC | (1 << BIT)>(kase, p, l, c, s, msign, g);
        else
            adj_dispatch<NEXT, ACC>(kase, p, l, c, s, msign, g);
    }
}

// HALF: half-tile transposes (anchored micro-groups), as in k_pass2.
template <typename Amp, int B, bool HALF>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_adj2(Amp *__restrict__ psi, Amp *__restrict__ lam, const double2 *__restrict__ coef, const PassArgs2 args,
       uint64_t ntiles, double *__restrict__ gpart)
{
    constexpr int NW = (1 << (B - kRegDims)) / 64;
    constexpr int LB = HALF ? B - 1 : B;
    extern __shared__ unsigned char lds_raw[];
    Amp *ldp = reinterpret_cast<Amp *>(lds_raw);
    Amp *ldl = ldp + (1 << LB);
    __shared__ double2 tab[kMaxRun];
    __shared__ double wacc[kMaxRun][NW];
    const uint32_t t = threadIdx.x;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) {
        const RotDesc2 &d = args.rot[t];
        const double2 cs = coef[d.k];
        double sv = args.inverse ? -cs.y : cs.y;
        if (d.flags & 2) sv = -sv;
        tab[t] = make_double2(cs.x, sv);
    }
    for (int i = t; i < kMaxRun * NW; i += blockDim.x) (&wacc[0][0])[i] = 0.0;
    uint32_t tsb = 0;
    for (int ri = 0; ri < nrot; ++ri) tsb |= (uint32_t)par32(t & args.rot[ri].zt) << ri;
    __syncthreads();
    uint64_t Lb0 = 0, LbL = 0;
    {
        const uint32_t b0 = deposit32(t, args.mg[0].npiv), bL = deposit32(t, args.mg[last].npiv);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if ((b0 >> i) & 1) Lb0 ^= args.v[i];
            if ((bL >> i) & 1) LbL ^= args.v[i];
        }
    }
#pragma unroll 1
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(coset_of(tile, args.xrot, ntiles), args.outer_mask);
        double2 p[kRegs], l[kRegs];
        {
            const uint64_t y0 = tb ^ Lb0;
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                p[j] = ld(psi[y0 ^ args.LU_first[j]]);
                l[j] = ld(lam[y0 ^ args.LU_first[j]]);
            }
        }
        uint32_t bprev = 0;
#pragma unroll 1
        for (int g = 0; g <= last; ++g) {
            const MGDesc2 &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const MGDesc2 &mp = args.mg[g - 1];
                if constexpr (HALF) {
                    const uint32_t lo = (1u << args.qbit) - 1;
                    const uint32_t bw = (bprev & lo) | ((bprev >> 1) & ~lo);
                    const uint32_t br = (bt & lo) | ((bt >> 1) & ~lo);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
#pragma unroll
                        for (int j = h; j < kRegs; j += 2) {
                            st(ldp[bw ^ mp.UC[j]], p[j]);
                            st(ldl[bw ^ mp.UC[j]], l[j]);
                        }
                        __syncthreads();
#pragma unroll
                        for (int j = h; j < kRegs; j += 2) {
                            p[j] = ld(ldp[br ^ m.UC[j]]);
                            l[j] = ld(ldl[br ^ m.UC[j]]);
                        }
                        __syncthreads();
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) {
                        st(ldp[bprev ^ mp.U[j]], p[j]);
                        st(ldl[bprev ^ mp.U[j]], l[j]);
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) {
                        p[j] = ld(ldp[bt ^ m.U[j]]);
                        l[j] = ld(ldl[bt ^ m.U[j]]);
                    }
                    __syncthreads();
                }
            }
            bprev = bt;
#pragma unroll 1
            for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                const RotDesc2 &d = args.rot[ri];
                const double2 cs = tab[ri];
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                double gr = 0.0;
                adj_dispatch<8, 0>(d.kase, p, l, cs.x, flip_if(cs.y, sg), d.msign, gr);
                gr = flip_if(gr, sg ^ ((uint32_t)d.flags >> 2));
                gr = wave_sum<64>(gr);
                // every lane holds the same wave sum and writes the same value:
                // no divergent branch inside the unstructured rotation loop
                wacc[ri][t >> 6] += gr;
            }
        }
        const uint64_t yL = tb ^ LbL;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            st(psi[yL ^ args.LU_last[j]], p[j]);
            st(lam[yL ^ args.LU_last[j]], l[j]);
        }
    }
    __syncthreads();
    if ((int)t < nrot) {
        double sum = 0.0;
        for (int w = 0; w < NW; ++w) sum += wacc[t][w];
        gpart[(uint64_t)blockIdx.x * kMaxRun + t] = sum;
    }
}

// One term on the registers: lam_j += sigma_j w beta psi_{j ^ CX} for every
// register j (beta = 1, or i when IMAG), sigma_j the register sign from msign.
template <int CX, bool IMAG>
__device__ __forceinline__ void ham_body(const double2 (&r)[kRegs], double2 (&l)[kRegs], double w, uint32_t msign)
{
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
        const double wj = flip_if(w, msign >> j);
        const double2 v = r[j ^ CX];
        if (IMAG) {
            l[j].x = fma(-wj, v.y, l[j].x);
            l[j].y = fma(wj, v.x, l[j].y);
        } else {
            l[j].x = fma(wj, v.x, l[j].x);
            l[j].y = fma(wj, v.y, l[j].y);
        }
    }
}

// Uniform branch tree over the partner mask (bits 3..0) and real/imaginary w.
template <int BIT, int ACC>
__device__ __forceinline__ void ham_dispatch(uint32_t cx, bool imag, const double2 (&r)[kRegs], double2 (&l)[kRegs],
                                             double w, uint32_t msign)
{
    if constexpr (BIT < 0) {
        if (imag)
            ham_body<ACC, true>(r, l, w, msign);
        else
            ham_body<ACC, false>(r, l, w, msign);
    } else {
        if (cx & (1u << BIT))
            ham_dispatch<BIT - 1, ACC | (1 << BIT)>(cx, imag, r, l, w, msign);
        else
            ham_dispatch<BIT - 1, ACC>(cx, imag, r, l, w, msign);
    }
}

// Persistent H psi pass (the adjoint's lam): psi and lam of a coset in
// registers, moved together through half-tile LDS buffers between
// micro-groups; lam (+)= sum_k w_k P_k psi over the pass's terms, lam read
// only when accumulating onto earlier passes.
template <typename Amp, int B>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_ham2(const Amp *__restrict__ psi, Amp *__restrict__ lam, const double2 *__restrict__ mw, const PassArgs2 args,
       uint64_t ntiles, int accumulate)
{
    constexpr int LB = B - 1;
    extern __shared__ unsigned char lds_raw[];
    Amp *ldp = reinterpret_cast<Amp *>(lds_raw);
    Amp *ldl = ldp + (1 << LB);
    __shared__ double2 tab[kMaxRun];
    const uint32_t t = threadIdx.x;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) tab[t] = mw[args.rot[t].k];
    uint32_t tsb = 0;
    for (int ri = 0; ri < nrot; ++ri) tsb |= (uint32_t)par32(t & args.rot[ri].zt) << ri;
    __syncthreads();
    uint64_t Lb0 = 0, LbL = 0;
    {
        const uint32_t b0 = deposit32(t, args.mg[0].npiv), bL = deposit32(t, args.mg[last].npiv);
#pragma unroll
        for (int i = 0; i < B; ++i) {
            if ((b0 >> i) & 1) Lb0 ^= args.v[i];
            if ((bL >> i) & 1) LbL ^= args.v[i];
        }
    }
#pragma unroll 1
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(coset_of(tile, args.xrot, ntiles), args.outer_mask);
        double2 p[kRegs], l[kRegs];
        {
            const uint64_t y0 = tb ^ Lb0;
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                p[j] = ld(psi[y0 ^ args.LU_first[j]]);
                l[j] = accumulate ? ld(lam[y0 ^ args.LU_first[j]]) : make_double2(0.0, 0.0);
            }
        }
        uint32_t bprev = 0;
#pragma unroll 1
        for (int g = 0; g <= last; ++g) {
            const MGDesc2 &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const MGDesc2 &mp = args.mg[g - 1];
                // bprev and bt have 0 at the anchor bit (it is a pivot)
                const uint32_t lo = (1u << args.qbit) - 1;
                const uint32_t bw = (bprev & lo) | ((bprev >> 1) & ~lo);
                const uint32_t br = (bt & lo) | ((bt >> 1) & ~lo);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int j = h; j < kRegs; j += 2) {
                        st(ldp[bw ^ mp.UC[j]], p[j]);
                        st(ldl[bw ^ mp.UC[j]], l[j]);
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = h; j < kRegs; j += 2) {
                        p[j] = ld(ldp[br ^ m.UC[j]]);
                        l[j] = ld(ldl[br ^ m.UC[j]]);
                    }
                    __syncthreads();
                }
            }
            bprev = bt;
#pragma unroll 1
            for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                const RotDesc2 &d = args.rot[ri];
                const double2 w = tab[ri];
                const bool imag = w.y != 0.0;
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                ham_dispatch<3, 0>(d.cx, imag, p, l, flip_if(imag ? w.y : w.x, sg), d.msign);
            }
        }
        const uint64_t yL = tb ^ LbL;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) st(lam[yL ^ args.LU_last[j]], l[j]);
    }
}

// grad[k of rotation ri] = sum over the pass's workgroups of their partials (fixed order).
__global__ void k_grad_reduce2(const double *__restrict__ gpart, int nblocks, const PassArgs2 args,
                               double *__restrict__ grad)
{
    const int ri = blockIdx.x;
    __shared__ double sh[256];
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) a += gpart[(uint64_t)b * kMaxRun + ri];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[args.rot[ri].k] = sh[0];
}

template <typename Amp, int B, bool HALF>
cfh_status launch_adj2_b(uint64_t ntiles, hipStream_t s, Amp *psi, Amp *lam, const double2 *coef,
                         const PassArgs2 &a, double *gpart, unsigned max_grid, double *grad)
{
    constexpr int LB = HALF ? B - 1 : B;
    if constexpr (2 * ((size_t)1 << LB) * sizeof(Amp) > 128 * 1024) {
        return set_error(CFH_E_UNSUPPORTED, "adjoint tile too large for LDS");
    } else {
        constexpr int T = 1 << (B - kRegDims);
        const size_t lds = a.nmg > 1 ? 2 * ((size_t)1 << LB) * sizeof(Amp) : 0;
        const void *fn = reinterpret_cast<const void *>(&k_adj2<Amp, B, HALF>);
        static std::atomic<bool> attr{false};  // LDS limit set once per kernel
        if (!attr.load(std::memory_order_acquire)) {
            hipFuncAttributes fa{};
            cfh_status st = CFH_OK;
            if (!hip_ok(hipFuncGetAttributes(&fa, fn), "k_adj2: hipFuncGetAttributes", &st)) return st;
            if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(160 * 1024 - fa.sharedSizeBytes)),
                        "k_adj2: hipFuncSetAttribute", &st))
                return st;
            attr.store(true, std::memory_order_release);
        }
        unsigned grid = (unsigned)std::min<uint64_t>(ntiles, resident_grid(fn, T, lds));
        grid = std::min(grid, max_grid);
        if (a.xrot > 0) grid &= ~7u;  // coset_of: one line group per XCD
        hipLaunchKernelGGL((k_adj2<Amp, B, HALF>), dim3(grid), dim3(T), lds, s, psi, lam, coef, a, ntiles, gpart);
        cfh_status st = last_launch("k_adj2");
        if (st) return st;
        const int nrot = a.mg[a.nmg - 1].rot_begin + a.mg[a.nmg - 1].rot_count;
        hipLaunchKernelGGL(k_grad_reduce2, dim3(nrot), dim3(256), 0, s, gpart, (int)grid, a, grad);
        return last_launch("k_grad_reduce2");
    }
}

template <typename Amp, int B, int MODE>
cfh_status launch_pass2_b(uint64_t ntiles, hipStream_t s, Amp *psi, const double2 *coef, const PassArgs2 &a,
                          double2 *partial, unsigned max_grid)
{
    constexpr int LB = (MODE & 4) ? B - 1 : B;  // log2 amplitudes in the transpose buffer
    if constexpr (((size_t)1 << LB) * sizeof(Amp) > 160 * 1024) {
        return set_error(CFH_E_UNSUPPORTED, "tile_bits too large for LDS");
    } else {
        constexpr int T = 1 << (B - kRegDims);
        const size_t lds = a.nmg > 1 ? ((size_t)1 << LB) * sizeof(Amp) : 0;
        const void *fn = reinterpret_cast<const void *>(&k_pass2<Amp, B, MODE>);
        static std::atomic<bool> attr{false};  // LDS limit set once per kernel
        if (!attr.load(std::memory_order_acquire)) {
            // dynamic LDS may take what the kernel's static LDS leaves of the 160 KiB
            hipFuncAttributes fa{};
            cfh_status st = CFH_OK;
            if (!hip_ok(hipFuncGetAttributes(&fa, fn), "k_pass2: hipFuncGetAttributes", &st)) return st;
            if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(160 * 1024 - fa.sharedSizeBytes)),
                        "k_pass2: hipFuncSetAttribute", &st))
                return st;
            attr.store(true, std::memory_order_release);
        }
        // read-only passes: four workgroups per resident slot, so workgroups
        // finish at different times and their load and term phases drift
        // apart (measured 2-4% faster than a resident grid)
        const uint64_t per = (MODE & 8) ? 4 : 1;
        unsigned grid = (unsigned)std::min<uint64_t>(ntiles, per * resident_grid(fn, T, lds));
        if (max_grid) grid = std::min(grid, max_grid);
        if (a.xrot > 0) grid &= ~7u;  // coset_of: one line group per XCD
        hipLaunchKernelGGL((k_pass2<Amp, B, MODE>), dim3(grid), dim3(T), lds, s, psi, coef, a, ntiles, partial);
        return last_launch("k_pass2");
    }
}

template <typename Amp, int B>
cfh_status launch_pass2_m(uint64_t ntiles, hipStream_t s, Amp *psi, const double2 *coef, const PassArgs2 &a, int mode,
                          double2 *partial, unsigned max_grid)
{
    switch (mode) {
    case 1: return launch_pass2_b<Amp, B, 1>(ntiles, s, psi, coef, a, partial, max_grid);
    case 18: return launch_pass2_b<Amp, B, 18>(ntiles, s, psi, coef, a, partial, max_grid);
    case 22: return launch_pass2_b<Amp, B, 22>(ntiles, s, psi, coef, a, partial, max_grid);
    case 10: return launch_pass2_b<Amp, B, 10>(ntiles, s, psi, coef, a, partial, max_grid);
    case 14: return launch_pass2_b<Amp, B, 14>(ntiles, s, psi, coef, a, partial, max_grid);
    default: return launch_pass2_b<Amp, B, 0>(ntiles, s, psi, coef, a, partial, max_grid);
    }
}

template <typename Amp, int B>
cfh_status launch_ham2_b(uint64_t ntiles, hipStream_t s, const Amp *psi, Amp *lam, const double2 *mw,
                         const PassArgs2 &a, int accumulate)
{
    if constexpr (2 * ((size_t)1 << (B - 1)) * sizeof(Amp) > 128 * 1024) {
        return set_error(CFH_E_UNSUPPORTED, "H psi tile too large for LDS");
    } else {
        constexpr int T = 1 << (B - kRegDims);
        const size_t lds = a.nmg > 1 ? 2 * ((size_t)1 << (B - 1)) * sizeof(Amp) : 0;
        const void *fn = reinterpret_cast<const void *>(&k_ham2<Amp, B>);
        static std::atomic<bool> attr{false};  // LDS limit set once per kernel
        if (!attr.load(std::memory_order_acquire)) {
            hipFuncAttributes fa{};
            cfh_status st = CFH_OK;
            if (!hip_ok(hipFuncGetAttributes(&fa, fn), "k_ham2: hipFuncGetAttributes", &st)) return st;
            if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(160 * 1024 - fa.sharedSizeBytes)),
                        "k_ham2: hipFuncSetAttribute", &st))
                return st;
            attr.store(true, std::memory_order_release);
        }
        unsigned grid = (unsigned)std::min<uint64_t>(ntiles, resident_grid(fn, T, lds));
        if (a.xrot > 0) grid &= ~7u;  // coset_of: one line group per XCD
        hipLaunchKernelGGL((k_ham2<Amp, B>), dim3(grid), dim3(T), lds, s, psi, lam, mw, a, ntiles, accumulate);
        return last_launch("k_ham2");
    }
}

} // namespace

namespace cfh {

template <typename Amp>
cfh_status launch_ham2(uint64_t ntiles, hipStream_t s, const Amp *psi, Amp *lam, const double2 *mw,
                       const PassArgs2 &a, int accumulate)
{
    switch (a.b) {
    case 10: return launch_ham2_b<Amp, 10>(ntiles, s, psi, lam, mw, a, accumulate);
    case 11: return launch_ham2_b<Amp, 11>(ntiles, s, psi, lam, mw, a, accumulate);
    case 12: return launch_ham2_b<Amp, 12>(ntiles, s, psi, lam, mw, a, accumulate);
    case 13: return launch_ham2_b<Amp, 13>(ntiles, s, psi, lam, mw, a, accumulate);
    default: return set_error(CFH_E_UNSUPPORTED, "register-tiled H psi needs tile_bits in 10..13");
    }
}

template <typename Amp>
cfh_status launch_adj2(uint64_t ntiles, hipStream_t s, Amp *psi, Amp *lam, const double2 *coef, const PassArgs2 &a,
                       bool half, double *gpart, unsigned max_grid, double *grad)
{
    switch (a.b) {
#define CFH_ADJ2_CASE(BB)                                                                                   \
    case BB:                                                                                                \
        return half ? launch_adj2_b<Amp, BB, true>(ntiles, s, psi, lam, coef, a, gpart, max_grid, grad)    \
                    : launch_adj2_b<Amp, BB, false>(ntiles, s, psi, lam, coef, a, gpart, max_grid, grad);
        CFH_ADJ2_CASE(10) CFH_ADJ2_CASE(11) CFH_ADJ2_CASE(12) CFH_ADJ2_CASE(13)
#undef CFH_ADJ2_CASE
    default:
        return set_error(CFH_E_UNSUPPORTED, "register-tiled adjoint needs tile_bits in 10..13");
    }
}

// Workgroups of 2^(b-4) threads: b >= 10 keeps them at one full wave or more.
template <typename Amp>
cfh_status launch_pass2(uint64_t ntiles, hipStream_t s, Amp *psi, const double2 *coef, const PassArgs2 &a, int mode,
                        double2 *partial, unsigned max_grid)
{
    switch (a.b) {
    case 10: return launch_pass2_m<Amp, 10>(ntiles, s, psi, coef, a, mode, partial, max_grid);
    case 11: return launch_pass2_m<Amp, 11>(ntiles, s, psi, coef, a, mode, partial, max_grid);
    case 12: return launch_pass2_m<Amp, 12>(ntiles, s, psi, coef, a, mode, partial, max_grid);
    case 13: return launch_pass2_m<Amp, 13>(ntiles, s, psi, coef, a, mode, partial, max_grid);
    case 14:
        // 1024-thread workgroups; only the half-tile transposes fit 2^14 complex128 in LDS
        if (mode == 22) return launch_pass2_b<Amp, 14, 22>(ntiles, s, psi, coef, a, partial, max_grid);
        if (mode == 14) return launch_pass2_b<Amp, 14, 14>(ntiles, s, psi, coef, a, partial, max_grid);
        return set_error(CFH_E_UNSUPPORTED, "tile_bits 14 needs the half-tile register-tiled kernel");
    default: return set_error(CFH_E_UNSUPPORTED, "register-tiled pass needs tile_bits in 10..14");
    }
}


} // namespace cfh
