// Register-tiled forward rotation passes of the batched runs (cfh_batch_*).
//
// Same scheme as the single-state register-tiled pass (k_pass2, compile-time
// pair bodies): a workgroup holds one coset of the pass's 2^b-amplitude tile
// subspace in registers, 16 amplitudes per thread, runs the pass's
// micro-groups with LDS transposes between them, and writes the coset back.
// Here every workgroup is one work item of a level: a range of cosets of one
// pass of one circuit, whose PassArgs2 sits in device memory.  The first pass
// of a circuit builds the initial basis state instead of reading psi.
#include "batch.hpp"
#include "pass2.hpp"

namespace {

template <typename Amp, int B>
__global__ void __launch_bounds__(1 << (B - kRegDims))
k_batch_fwd2(const BatchArgs A, const PassArgs2 *__restrict__ pa, const BItem *__restrict__ items)
{
    extern __shared__ unsigned char lds_raw[];
    Amp *lds = reinterpret_cast<Amp *>(lds_raw);
    __shared__ double2 tab[kMaxRun];
    const uint32_t t = threadIdx.x;
    const BItem it = items[blockIdx.x];
    const BPass &P = A.passes[it.pass];
    const BCirc &C = A.circs[P.circ];
    const PassArgs2 &args = pa[P.p2];
    Amp *psi = reinterpret_cast<Amp *>(A.psi) + C.psi_off;
    const double2 *coef = A.coef + C.theta_off;
    const int last = args.nmg - 1;
    const int nrot = args.mg[last].rot_begin + args.mg[last].rot_count;
    if ((int)t < nrot) {
        const RotDesc2 &d = args.rot[t];
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
            const MGDesc2 &m = args.mg[g];
            const uint32_t bt = deposit32(t, m.npiv);
            if (g > 0) {
                const MGDesc2 &mp = args.mg[g - 1];
#pragma unroll
                for (int j = 0; j < kRegs; ++j) st(lds[bprev ^ mp.U[j]], r[j]);
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kRegs; ++j) r[j] = ld(lds[bt ^ m.U[j]]);
                __syncthreads();
            }
            bprev = bt;
#pragma unroll 1
            for (int ri = m.rot_begin; ri < m.rot_begin + m.rot_count; ++ri) {
                const RotDesc2 &d = args.rot[ri];
                const double2 cs = tab[ri];
                const uint32_t sg = ((tsb >> ri) ^ (uint32_t)par64(tb & d.z)) & 1u;
                kase_dispatch<8, 0>(d.kase, r, cs.x, flip_if(cs.y, sg));
            }
        }
        const uint64_t yL = tb ^ LbL;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) st(psi[yL ^ args.LU_last[j]], r[j]);
    }
}

} // namespace

namespace cfh {

template <typename Amp>
cfh_status launch_batch_fwd2(unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items)
{
    constexpr int B = kBatchRegTile;
    constexpr int T = 1 << (B - kRegDims);
    constexpr size_t lds = ((size_t)1 << B) * sizeof(Amp);
    const void *fn = reinterpret_cast<const void *>(&k_batch_fwd2<Amp, B>);
    static bool attr = false;
    if (!attr) {
        hipFuncAttributes fa{};
        cfh_status st = CFH_OK;
        if (!hip_ok(hipFuncGetAttributes(&fa, fn), "k_batch_fwd2: hipFuncGetAttributes", &st)) return st;
        if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(160 * 1024 - fa.sharedSizeBytes)),
                    "k_batch_fwd2: hipFuncSetAttribute", &st))
            return st;
        attr = true;
    }
    hipLaunchKernelGGL((k_batch_fwd2<Amp, B>), dim3(grid), dim3(T), lds, s, A, pa, items);
    return last_launch("k_batch_fwd2");
}

template cfh_status launch_batch_fwd2<double2>(unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                               const BItem *);
template cfh_status launch_batch_fwd2<float2>(unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                              const BItem *);

} // namespace cfh
