// Register-tiled forward, adjoint, measurement and H psi passes of the
// batched runs (cfh_batch_*).
//
// Same scheme as the single-state register-tiled pass (k_pass2, compile-time
// pair bodies): a workgroup holds one coset of the pass's 2^b-amplitude tile
// subspace in registers, 16 amplitudes per thread, runs the pass's
// micro-groups with LDS transposes between them, and writes the coset back.
// Here every workgroup is one work item of a level: a range of cosets of one
// pass of one circuit, whose PassArgs2 sits in device memory.  The first pass
// of a circuit builds the initial basis state instead of reading psi.
#include <atomic>

#include "batch.hpp"
#include "pass2.hpp"

namespace {

// The pass, circuit and kernel descriptor tables are written by the host
// before a run and only read by its kernels: reads through the constant
// address space let uniform ones use scalar loads, also after the fences of
// a persistent workgroup's loop.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T &cref(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

template <typename Amp, int B, bool HALF>
__device__ __forceinline__ void fwd2_item(const BatchArgs &A, const PassArgs2 *__restrict__ pa, const BItem it,
                                          unsigned char *lds_raw)
{
    Amp *lds = reinterpret_cast<Amp *>(lds_raw);
    __shared__ double2 tab[kMaxRun];
    const uint32_t t = threadIdx.x;
    const auto &P = cref(A.passes + it.pass);
    const auto &C = cref(A.circs + P.circ);
    const auto &args = cref(pa + P.p2);
    Amp *psi = reinterpret_cast<Amp *>(A.psi) + C.psi_off;
    const double2 *coef = A.coef + C.theta_off;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) {
        const auto &d = args.rot[t];
        const double2 cs = coef[d.k];
        tab[t] = make_double2(cs.x, (d.flags & 2) ? -cs.y : cs.y);
    }
    uint32_t tsb = 0;  // bit ri: parity(t & zt) of rotation ri
    for (int ri = 0; ri < nrot; ++ri) tsb |= (uint32_t)par32(t & args.rot[ri].zt) << ri;
    if ((P.flags & kFlagStart) && it.idx == 0 && t == 0) A.t_start[P.circ] = wall_clock64();
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
    const bool init = P.flags & kFlagInit;
    const uint64_t ntiles = 1ull << (C.n - args.b);
    const uint64_t tile0 = (uint64_t)it.idx * (uint64_t)P.tiles_per_item;
    const uint64_t tile1 = std::min<uint64_t>(ntiles, tile0 + (uint64_t)P.tiles_per_item);
#pragma unroll 1
    for (uint64_t tile = tile0; tile < tile1; ++tile) {
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(tile, args.outer_mask);
        double2 r[kRegs];
        const uint64_t y0 = tb ^ Lb0;
        if (init) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) r[j] = make_double2((y0 ^ args.LU_first[j]) == C.init ? 1.0 : 0.0, 0.0);
        } else {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) r[j] = ld(psi[y0 ^ args.LU_first[j]]);
        }
        uint32_t bprev = 0;
#pragma unroll 1
        for (int g = 0; g <= last; ++g) {
            const auto &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const auto &mp = args.mg[g - 1];
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
#pragma unroll 1
            for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                const auto &d = args.rot[ri];
                const double2 cs = tab[ri];
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                kase_switch(d.kase, r, cs.x, flip_if(cs.y, sg));
            }
        }
        const uint64_t yL = tb ^ LbL;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) st(psi[yL ^ args.LU_last[j]], r[j]);
    }
}

// Adjoint items: psi and lam of a coset in registers, the pass's rotations
// walked backwards (inverse-order descriptors, half-tile transposes of both
// vectors), each rotation's share of g_k = Im <lam|P_k|psi> summed per wave
// over the item's cosets and written to the item's gradient partials, which
// the level's reduction adds in a fixed order.
template <typename Amp, int B, bool HALF>
__device__ __forceinline__ void adj2_item(const BatchArgs &A, const PassArgs2 *__restrict__ pa, const BItem it,
                                          unsigned char *lds_raw)
{
    constexpr int NW = (1 << (B - kRegDims)) / 64;
    constexpr int LB = HALF ? B - 1 : B;
    Amp *ldp = reinterpret_cast<Amp *>(lds_raw);
    Amp *ldl = ldp + (1 << LB);
    __shared__ double2 tab[kMaxRun];
    __shared__ double wacc[kMaxRun][NW];
    const uint32_t t = threadIdx.x;
    const auto &P = cref(A.passes + it.pass);
    const auto &C = cref(A.circs + P.circ);
    const auto &args = cref(pa + P.p2);
    Amp *psi = reinterpret_cast<Amp *>(A.psi) + C.psi_off;
    Amp *lam = reinterpret_cast<Amp *>(A.lam) + C.psi_off;
    const double2 *coef = A.coef + C.theta_off;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) {
        const auto &d = args.rot[t];
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
    const uint64_t ntiles = 1ull << (C.n - args.b);
    const uint64_t tile0 = (uint64_t)it.idx * (uint64_t)P.tiles_per_item;
    const uint64_t tile1 = std::min<uint64_t>(ntiles, tile0 + (uint64_t)P.tiles_per_item);
#pragma unroll 1
    for (uint64_t tile = tile0; tile < tile1; ++tile) {
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(tile, args.outer_mask);
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
            const auto &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const auto &mp = args.mg[g - 1];
                if constexpr (HALF) {
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
                const auto &d = args.rot[ri];
                const double2 cs = tab[ri];
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                double gr = 0.0;
                adj_dispatch<8, 0>(d.kase, p, l, cs.x, flip_if(cs.y, sg), d.msign, gr);
                gr = flip_if(gr, sg ^ ((uint32_t)d.flags >> 2));
                gr = wave_sum<64>(gr);
                // every lane holds the same wave sum and writes the same value
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
        A.gpart[C.gpart_off + (int64_t)it.idx * kMaxRun + t] = sum;
    }
}

// Measurement items: the terms of the pass on the coset's registers, read
// only (the single-state measurement pass, per work item); complex128 items
// transpose in two halves through half the LDS, as the forward items do.
template <typename Amp, int B, bool HALF>
__device__ __forceinline__ void meas2_item(const BatchArgs &A, const PassArgs2 *__restrict__ pa, const BItem it,
                                           unsigned char *lds_raw)
{
    constexpr int NW = (1 << (B - kRegDims)) / 64;
    Amp *lds = reinterpret_cast<Amp *>(lds_raw);
    __shared__ double2 tab[kMaxRun];
    __shared__ double red[NW];
    const uint32_t t = threadIdx.x;
    const auto &P = cref(A.passes + it.pass);
    const auto &C = cref(A.circs + P.circ);
    const auto &args = cref(pa + P.p2);
    const Amp *psi = reinterpret_cast<const Amp *>(A.psi) + C.psi_off;
    const double2 *mw = A.mw + C.mw_off;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) tab[t] = mw[args.rot[t].k];
    uint32_t tsb = 0;
    for (int ri = 0; ri < nrot; ++ri) tsb |= (uint32_t)par32(t & args.rot[ri].zt) << ri;
    __syncthreads();
    uint64_t Lb0 = 0;
    {
        const uint32_t b0 = deposit32(t, args.mg[0].npiv);
#pragma unroll
        for (int i = 0; i < B; ++i)
            if ((b0 >> i) & 1) Lb0 ^= args.v[i];
    }
    double accr = 0.0, acci = 0.0;
    const uint64_t ntiles = 1ull << (C.n - args.b);
    const uint64_t tile0 = (uint64_t)it.idx * (uint64_t)P.tiles_per_item;
    const uint64_t tile1 = std::min<uint64_t>(ntiles, tile0 + (uint64_t)P.tiles_per_item);
#pragma unroll 1
    for (uint64_t tile = tile0; tile < tile1; ++tile) {
        asm volatile("" : "+v"(Lb0));
        const uint64_t tb = deposit(tile, args.outer_mask);
        double2 r[kRegs];
        const uint64_t y0 = tb ^ Lb0;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) r[j] = ld(psi[y0 ^ args.LU_first[j]]);
        uint32_t bprev = 0;
#pragma unroll 1
        for (int g = 0; g <= last; ++g) {
            const auto &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const auto &mp = args.mg[g - 1];
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
#pragma unroll 1
            for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                // the amplitudes do not change between terms: keep the products
                // of all partner masks from being hoisted out of the loop
#pragma unroll
                for (int j = 0; j < kRegs; ++j) asm volatile("" : "+v"(r[j].x), "+v"(r[j].y));
                const auto &d = args.rot[ri];
                const double2 w = tab[ri];
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                meas_switch(d.kase, r, flip_if(w.x, sg), flip_if(w.y, sg), accr, acci);
            }
        }
    }
    accr = wave_sum<64>(accr);
    if ((t & 63) == 0) red[t >> 6] = accr;
    __syncthreads();
    if (t == 0) {
        double sr = 0.0;
        for (int i = 0; i < NW; ++i) sr += red[i];
        double *slot = A.epart + C.epart_off + it.idx;
        // written by item it.idx of the circuit's previous measurement pass,
        // possibly on another XCD in a persistent run: a vector load at agent scope
        *slot = (P.flags & kFlagAccumulate)
                    ? __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + sr
                    : sr;
    }
}

// H psi items (gradient runs): psi and lam of a coset in registers (half-tile
// transposes of both), lam += sum_k w_k P_k psi over the pass's terms (lam
// starts at zero on the circuit's first such pass), lam written back; the
// last pass also adds Re <psi|lam> over the item's cosets to its energy
// partial.
template <typename Amp, int B, bool HALF>
__device__ __forceinline__ void ham2_item(const BatchArgs &A, const PassArgs2 *__restrict__ pa, const BItem it,
                                          unsigned char *lds_raw)
{
    constexpr int NW = (1 << (B - kRegDims)) / 64;
    constexpr int LB = HALF ? B - 1 : B;
    Amp *ldp = reinterpret_cast<Amp *>(lds_raw);
    Amp *ldl = ldp + (1 << LB);
    __shared__ double2 tab[kMaxRun];
    __shared__ double red[NW];
    const uint32_t t = threadIdx.x;
    const auto &P = cref(A.passes + it.pass);
    const auto &C = cref(A.circs + P.circ);
    const auto &args = cref(pa + P.p2);
    const Amp *psi = reinterpret_cast<const Amp *>(A.psi) + C.psi_off;
    Amp *lam = reinterpret_cast<Amp *>(A.lam) + C.psi_off;
    const double2 *mw = A.mw + C.mw_off;
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
    const bool accumulate = P.flags & kFlagAccumulate;
    const bool energy = P.flags & kFlagEnergy;
    double eacc = 0.0;
    const uint64_t ntiles = 1ull << (C.n - args.b);
    const uint64_t tile0 = (uint64_t)it.idx * (uint64_t)P.tiles_per_item;
    const uint64_t tile1 = std::min<uint64_t>(ntiles, tile0 + (uint64_t)P.tiles_per_item);
#pragma unroll 1
    for (uint64_t tile = tile0; tile < tile1; ++tile) {
        asm volatile("" : "+v"(Lb0), "+v"(LbL));
        const uint64_t tb = deposit(tile, args.outer_mask);
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
            const auto &m = args.mg[g];
            const uint32_t bt = deposit_tid(t, m.npiv);
            if (g > 0) {
                const auto &mp = args.mg[g - 1];
                if constexpr (HALF) {
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
                const auto &d = args.rot[ri];
                const double2 w = tab[ri];
                const bool imag = w.y != 0.0;
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                ham_dispatch<3, 0>(d.cx, imag, p, l, flip_if(imag ? w.y : w.x, sg), d.msign);
            }
        }
        const uint64_t yL = tb ^ LbL;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            st(lam[yL ^ args.LU_last[j]], l[j]);
            if (energy) {
                Amp stored;  // lam as stored (rounded to the storage type)
                st(stored, l[j]);
                const double2 o = ld(stored);
                eacc += p[j].x * o.x + p[j].y * o.y;
            }
        }
    }
    if (energy) {
        eacc = wave_sum<64>(eacc);
        if ((t & 63) == 0) red[t >> 6] = eacc;
        __syncthreads();
        if (t == 0) {
            double sr = 0.0;
            for (int i = 0; i < NW; ++i) sr += red[i];
            A.epart[C.epart_off + it.idx] = sr;
        }
    }
}

// One work item per workgroup: the level-synchronous kernels.
template <typename Amp, int B, bool HALF>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_fwd2(const BatchArgs A, const PassArgs2 *__restrict__ pa, const BItem *__restrict__ items)
{
    extern __shared__ unsigned char lds_raw[];
    fwd2_item<Amp, B, HALF>(A, pa, items[blockIdx.x], lds_raw);
}

template <typename Amp, int B, bool HALF>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_adj2(const BatchArgs A, const PassArgs2 *__restrict__ pa, const BItem *__restrict__ items)
{
    extern __shared__ unsigned char lds_raw[];
    adj2_item<Amp, B, HALF>(A, pa, items[blockIdx.x], lds_raw);
}

template <typename Amp, int B, bool HALF>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_meas2(const BatchArgs A, const PassArgs2 *__restrict__ pa, const BItem *__restrict__ items)
{
    extern __shared__ unsigned char lds_raw[];
    meas2_item<Amp, B, HALF>(A, pa, items[blockIdx.x], lds_raw);
}

template <typename Amp, int B, bool HALF>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_ham2(const BatchArgs A, const PassArgs2 *__restrict__ pa, const BItem *__restrict__ items)
{
    extern __shared__ unsigned char lds_raw[];
    ham2_item<Amp, B, HALF>(A, pa, items[blockIdx.x], lds_raw);
}

// Wait until *flag >= need.  Thread 0 of a workgroup polls with agent-scope
// loads (they bypass the XCD's own L2, so a store from any XCD is seen),
// sleeping between polls.  It gives up after max_ticks of the constant-rate
// wall clock (100 MHz), or as soon as another workgroup has given up; as a
// backstop that does not rely on the clock, also after max_ticks / 8 polls
// (a poll's sleep alone, 256 shader clocks, outlasts 8 ticks, so this bound
// lies beyond the clock's).  A workgroup that gives up raises the abort word
// and the status word.
__device__ bool wait_ready(const uint32_t *flag, uint32_t need, uint32_t *ctl, uint64_t max_ticks)
{
    const uint64_t t0 = wall_clock64();
    const uint64_t max_polls = max_ticks / 8 + 1;
    for (uint64_t polls = 0;; ++polls) {
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return true;
        if (__hip_atomic_load(&ctl[kCtlAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (polls >= max_polls || wall_clock64() - t0 >= max_ticks) {
            __hip_atomic_store(&ctl[kCtlStatus], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl[kCtlAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// Persistent dataflow schedule: a grid of resident workgroups takes tickets
// from one counter.  Ticket k is a work item; the ticket table lists every
// item after all items of the pass before it in its circuit's chain, so an
// item's only dependency is that one pass.  A workgroup waits until that
// pass is ready, runs the item, publishes its stores (release), and counts
// the item done; the workgroup that finishes a pass's last item reduces the
// pass's partial sums (the level kernels' fixed order) and then marks the
// pass ready.  Tickets are claimed in table order and only by running
// workgroups, so the smallest unfinished claimed ticket always has its
// dependency finished: the schedule completes whatever the number of
// workgroups the device keeps resident.  A workgroup whose wait gives up
// leaves, so a run that cannot finish still ends.
template <typename Amp, int B, bool GRAD>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_persist(const BatchArgs A, const PassArgs2 *__restrict__ pa, const PersistArgs Q)
{
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    extern __shared__ unsigned char lds_raw[];
    __shared__ int s_ticket, s_last;
    __shared__ double sh[kBThreads];
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) {
            int tk = -1;
            if (__hip_atomic_load(&Q.ctl[kCtlAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
                tk = (int)__hip_atomic_fetch_add(&Q.ctl[kCtlTicket], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tk >= Q.nt) tk = -1;
            if (tk >= 0) {
                const int pp = Q.prev[Q.tickets[tk].pass];
                if (pp >= 0 && !wait_ready(&Q.ready[pp], Q.need, Q.ctl, Q.max_wait)) tk = -1;
            }
            // acquire at agent scope once per item, for the whole workgroup:
            // the barrier below orders every wave's reads after it
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ticket = tk;
        }
        __syncthreads();
        // the same ticket in every lane: uniform, so its descriptors load into scalar registers
        const int tk = __builtin_amdgcn_readfirstlane(s_ticket);
        if (tk < 0) return;
        const BItem it = {cref(Q.tickets + tk).pass, cref(Q.tickets + tk).idx};
        const int ty = cref(A.passes + it.pass).type;
        if (ty == kPassFwd) {
            fwd2_item<Amp, B, HALF>(A, pa, it, lds_raw);
        } else if constexpr (GRAD) {
            if (ty == kPassHam)
                ham2_item<Amp, B, HALF>(A, pa, it, lds_raw);
            else if (ty == kPassAdj)
                adj2_item<Amp, B, HALF>(A, pa, it, lds_raw);
        } else {
            if (ty == kPassMeas) meas2_item<Amp, B, HALF>(A, pa, it, lds_raw);
        }
        // the barrier orders every wave's stores before thread 0's count,
        // whose agent-scope release publishes them device-wide (one write-back
        // per item); its acquire half lets the pass's last item see the others
        __syncthreads();
        if (t == 0) {
            const uint32_t before =
                __hip_atomic_fetch_add(&Q.done[it.pass], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_last = before + 1 == (uint32_t)cref(A.passes + it.pass).nitems;
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_last)) {
            reduce_pass(A, it.pass, sh);
            __syncthreads();
            if (t == 0) __hip_atomic_store(&Q.ready[it.pass], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

template <typename KernelFn>
cfh_status set_lds_limit(KernelFn fn, const char *what)
{
    hipFuncAttributes fa{};
    cfh_status st = CFH_OK;
    if (!hip_ok(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(fn)), what, &st)) return st;
    hip_ok(hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(160 * 1024 - fa.sharedSizeBytes)),
           what, &st);
    return st;
}

} // namespace

namespace cfh {

template <typename Amp, int B>
cfh_status launch_batch_fwd2_b(unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    constexpr int T = 1 << (B - kRegDims);
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    constexpr size_t lds = ((size_t)1 << (HALF ? B - 1 : B)) * sizeof(Amp);
    static std::atomic<bool> attr{false};  // LDS limit set once per kernel
    if (!attr.load(std::memory_order_acquire)) {
        if (cfh_status st = set_lds_limit(&k_batch_fwd2<Amp, B, HALF>, "k_batch_fwd2: LDS limit")) return st;
        attr.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL((k_batch_fwd2<Amp, B, HALF>), dim3(grid), dim3(T), lds, s, A, pa, items);
    return last_launch("k_batch_fwd2");
}

template <typename Amp, int B>
cfh_status launch_batch_meas2_b(unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                              const BItem *items)
{
    constexpr int T = 1 << (B - kRegDims);
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    constexpr size_t lds = ((size_t)1 << (HALF ? B - 1 : B)) * sizeof(Amp);
    static std::atomic<bool> attr{false};  // LDS limit set once per kernel
    if (!attr.load(std::memory_order_acquire)) {
        if (cfh_status st = set_lds_limit(&k_batch_meas2<Amp, B, HALF>, "k_batch_meas2: LDS limit")) return st;
        attr.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL((k_batch_meas2<Amp, B, HALF>), dim3(grid), dim3(T), lds, s, A, pa, items);
    return last_launch("k_batch_meas2");
}

template <typename Amp, int B>
cfh_status launch_batch_ham2_b(unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    constexpr int T = 1 << (B - kRegDims);
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    // psi and lam buffers: half tiles at complex128, whole tiles at complex64
    constexpr size_t lds = 2 * ((size_t)1 << (HALF ? B - 1 : B)) * sizeof(Amp);
    static std::atomic<bool> attr{false};  // LDS limit set once per kernel
    if (!attr.load(std::memory_order_acquire)) {
        if (cfh_status st = set_lds_limit(&k_batch_ham2<Amp, B, HALF>, "k_batch_ham2: LDS limit")) return st;
        attr.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL((k_batch_ham2<Amp, B, HALF>), dim3(grid), dim3(T), lds, s, A, pa, items);
    return last_launch("k_batch_ham2");
}

template <typename Amp, int B>
cfh_status launch_batch_adj2_b(unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    constexpr int T = 1 << (B - kRegDims);
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    // psi and lam buffers: half tiles at complex128, whole tiles at complex64
    constexpr size_t lds = 2 * ((size_t)1 << (HALF ? B - 1 : B)) * sizeof(Amp);
    static std::atomic<bool> attr{false};  // LDS limit set once per kernel
    if (!attr.load(std::memory_order_acquire)) {
        if (cfh_status st = set_lds_limit(&k_batch_adj2<Amp, B, HALF>, "k_batch_adj2: LDS limit")) return st;
        attr.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL((k_batch_adj2<Amp, B, HALF>), dim3(grid), dim3(T), lds, s, A, pa, items);
    return last_launch("k_batch_adj2");
}

template <typename Amp>
cfh_status launch_batch_fwd2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    switch (reg_bits) {
    case 11: return launch_batch_fwd2_b<Amp, 11>(grid, s, A, pa, items);
    case 12: return launch_batch_fwd2_b<Amp, 12>(grid, s, A, pa, items);
    case 13: return launch_batch_fwd2_b<Amp, 13>(grid, s, A, pa, items);
    default: return set_error(CFH_E_UNSUPPORTED, "batched register tile must be 2^11..2^13");
    }
}

template <typename Amp>
cfh_status launch_batch_meas2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    switch (reg_bits) {
    case 11: return launch_batch_meas2_b<Amp, 11>(grid, s, A, pa, items);
    case 12: return launch_batch_meas2_b<Amp, 12>(grid, s, A, pa, items);
    case 13: return launch_batch_meas2_b<Amp, 13>(grid, s, A, pa, items);
    default: return set_error(CFH_E_UNSUPPORTED, "batched register tile must be 2^11..2^13");
    }
}

template <typename Amp>
cfh_status launch_batch_ham2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    switch (reg_bits) {
    case 11: return launch_batch_ham2_b<Amp, 11>(grid, s, A, pa, items);
    case 12: return launch_batch_ham2_b<Amp, 12>(grid, s, A, pa, items);
    case 13: return launch_batch_ham2_b<Amp, 13>(grid, s, A, pa, items);
    default: return set_error(CFH_E_UNSUPPORTED, "batched register tile must be 2^11..2^13");
    }
}

template <typename Amp>
cfh_status launch_batch_adj2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    switch (reg_bits) {
    case 11: return launch_batch_adj2_b<Amp, 11>(grid, s, A, pa, items);
    case 12: return launch_batch_adj2_b<Amp, 12>(grid, s, A, pa, items);
    case 13: return launch_batch_adj2_b<Amp, 13>(grid, s, A, pa, items);
    default: return set_error(CFH_E_UNSUPPORTED, "batched register tile must be 2^11..2^13");
    }
}

// Dynamic LDS of a persistent workgroup: the largest of its item kinds.
// Forward runs (rotation and measurement items) hold one tile, halved at
// complex128; gradient runs (H psi and adjoint items) hold psi and lam.
template <typename Amp, int B, bool GRAD>
constexpr size_t persist_lds()
{
    constexpr bool HALF = batch_fwd_half((int)sizeof(Amp));
    constexpr size_t tile = ((size_t)1 << (HALF ? B - 1 : B)) * sizeof(Amp);
    return GRAD ? 2 * tile : tile;
}

template <typename Amp, int B, bool GRAD>
cfh_status launch_batch_persist_b(int max_grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                                  const PersistArgs &Q, int *grid_out)
{
    constexpr int T = 1 << (B - kRegDims);
    constexpr size_t lds = persist_lds<Amp, B, GRAD>();
    auto kern = &k_batch_persist<Amp, B, GRAD>;
    static std::atomic<bool> attr{false};  // LDS limit set once per kernel
    if (!attr.load(std::memory_order_acquire)) {
        if (cfh_status st = set_lds_limit(kern, "k_batch_persist: LDS limit")) return st;
        attr.store(true, std::memory_order_release);
    }
    // the current device's CUs and the workgroups of this kernel that fit on one
    int per_cu = 0, cus = 0, dev = 0;
    cfh_status st = CFH_OK;
    if (!hip_ok(hipGetDevice(&dev), "k_batch_persist: hipGetDevice", &st) ||
        !hip_ok(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "k_batch_persist: CUs", &st) ||
        !hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), T, lds),
                "k_batch_persist: occupancy", &st))
        return st;
    if (per_cu < 1 || cus < 1) return set_error(CFH_E_HIP, "k_batch_persist: no resident workgroup fits a CU");
    // by default the workgroups the occupancy calculation says fit at once;
    // any other grid also completes (items go only to running workgroups)
    int grid = max_grid > 0 ? max_grid : per_cu * cus;
    grid = std::max(1, std::min(grid, Q.nt));
    if (grid_out) *grid_out = grid;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(T), lds, s, A, pa, Q);
    return last_launch("k_batch_persist");
}

template <typename Amp>
cfh_status launch_batch_persist(int reg_bits, bool grad, int max_grid, hipStream_t s, const BatchArgs &A,
                                const PassArgs2 *pa, const PersistArgs &Q, int *grid_out)
{
    switch (reg_bits * 2 + (grad ? 1 : 0)) {
    case 22: return launch_batch_persist_b<Amp, 11, false>(max_grid, s, A, pa, Q, grid_out);
    case 23: return launch_batch_persist_b<Amp, 11, true>(max_grid, s, A, pa, Q, grid_out);
    case 24: return launch_batch_persist_b<Amp, 12, false>(max_grid, s, A, pa, Q, grid_out);
    case 25: return launch_batch_persist_b<Amp, 12, true>(max_grid, s, A, pa, Q, grid_out);
    case 26: return launch_batch_persist_b<Amp, 13, false>(max_grid, s, A, pa, Q, grid_out);
    case 27: return launch_batch_persist_b<Amp, 13, true>(max_grid, s, A, pa, Q, grid_out);
    default: return set_error(CFH_E_UNSUPPORTED, "batched register tile must be 2^11..2^13");
    }
}

template cfh_status launch_batch_persist<double2>(int, bool, int, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                  const PersistArgs &, int *);
template cfh_status launch_batch_persist<float2>(int, bool, int, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                 const PersistArgs &, int *);
template cfh_status launch_batch_fwd2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_fwd2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_meas2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_meas2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_ham2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_ham2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_adj2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);
template cfh_status launch_batch_adj2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                             const BItem *);

} // namespace cfh
