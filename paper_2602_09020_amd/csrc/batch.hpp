// Host and device layout of the batched runs (cfh_batch_*), shared by the
// LDS-staged level kernel and the register-tiled forward kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cfh_internal.hpp"

namespace cfh {

constexpr int kBThreads = 256;
constexpr int kBWaves = kBThreads / 64;

enum { kPassFwd = 0, kPassHam = 1, kPassAdj = 2, kPassMeas = 3 };
// Kernels that run a level's work items.
enum { kKernLds = 0, kKernFwd2 = 1, kKernAdj2 = 2, kKernMeas2 = 3, kKernHam2 = 4, kKernCount = 5 };
enum { kFlagInit = 1, kFlagAccumulate = 2, kFlagEnergy = 4, kFlagStart = 8, kFlagEnd = 16 };

struct BPass {
    uint64_t outer_mask;
    uint64_t v[kMaxTileBits];
    int32_t type, circ, b, flags;
    int32_t nitems;      // work items of this pass
    int32_t tiles_per_item;
    int32_t first;       // first rotation (fwd/adj) or group (ham) in the batch arrays
    int32_t count;       // number of rotations / groups
    int32_t end_flag_grad;  // 1 if this pass ends the circuit in a gradient run
    int32_t p2;          // register-tiled forward pass: index of its PassArgs2, else -1
    int32_t pad[2];
};

struct BCirc {
    int64_t psi_off;     // amplitude offset of the circuit's state in the arenas
    uint64_t init;       // initial basis index
    int64_t theta_off;   // offset of its angles / gradients
    int64_t gpart_off;   // per-item gradient partials (items * kMaxRun doubles)
    int64_t epart_off;   // per-item energy partials (items doubles)
    int64_t mw_off;      // its observable's term weights c_k i^{(e-|x&z|)} (measurement passes)
    int32_t n, pad;
};

struct BItem {
    int32_t pass;
    int32_t idx;         // item index inside its pass
};

struct BatchArgs {
    const BPass *passes;
    const BCirc *circs;
    const RotDesc *rot;
    const HamGroupDev *groups;
    const HamTermDev *terms;
    const double2 *coef;
    const double2 *mw;
    void *psi;
    void *lam;
    double *grad;
    double *energy;
    double *gpart;
    double *epart;
    uint64_t *t_start;
    uint64_t *t_end;
    int with_grad;
    int pad;
};

// Register-tiled forward rotation items of one level: one workgroup of
// 2^(b-4) threads per item, every item a range of cosets of one pass whose
// PassArgs2 is pa[passes[item.pass].p2].  The first pass of a circuit builds
// its basis state instead of reading psi.
constexpr int kBatchRegTile = 12;  // default register tile (tuning reg_tile_bits)
// Complex128 items transpose in two halves through half the LDS (anchored
// micro-groups), so as many workgroups fit on a CU as complex64 ones do with
// whole-tile transposes.
constexpr bool batch_fwd_half(int amp_bytes) { return amp_bytes == 16; }
template <typename Amp>
cfh_status launch_batch_fwd2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items);
extern template cfh_status launch_batch_fwd2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                      const BItem *);
extern template cfh_status launch_batch_fwd2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                     const BItem *);

// Register-tiled read-only measurement items (forward runs): each adds its
// share of sum_k w_k <psi|P_k|psi> over its cosets to its energy partial
// (assigned by the first measurement pass of the circuit, added by the rest).
template <typename Amp>
cfh_status launch_batch_meas2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                              const BItem *items);
extern template cfh_status launch_batch_meas2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                       const BItem *);
extern template cfh_status launch_batch_meas2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                      const BItem *);

// Register-tiled H psi items (gradient runs): lam (+)= sum_k w_k P_k psi on
// the pass's terms; the circuit's last such pass also writes the energy
// partials Re <psi|lam> of its items.
template <typename Amp>
cfh_status launch_batch_ham2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items);
extern template cfh_status launch_batch_ham2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                      const BItem *);
extern template cfh_status launch_batch_ham2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                     const BItem *);

// Register-tiled adjoint items of one level (half-tile transposes of psi and
// lam): gradient partials per item as the LDS-staged adjoint items write them.
template <typename Amp>
cfh_status launch_batch_adj2(int reg_bits, unsigned grid, hipStream_t s, const BatchArgs &A, const PassArgs2 *pa,
                             const BItem *items);
extern template cfh_status launch_batch_adj2<double2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                      const BItem *);
extern template cfh_status launch_batch_adj2<float2>(int, unsigned, hipStream_t, const BatchArgs &, const PassArgs2 *,
                                                     const BItem *);

} // namespace cfh
