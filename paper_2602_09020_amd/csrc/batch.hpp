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

// Fixed-order reduction of one finished pass's per-item partial sums, run by
// one workgroup (any size): gradient slot r of an adjoint pass is split over
// kBThreads / kMaxRun item lanes, each lane a strided share of the items,
// and the lane sums are added in a fixed order; an energy pass's item
// partials likewise.  The circuit's end stamp is taken when its last pass is
// reduced.  Every schedule reduces this way, so results are bitwise
// reproducible and equal across schedules.  sh holds kBThreads doubles.
__device__ inline void reduce_pass(const BatchArgs &A, int p, double *sh)
{
    constexpr int LANES = kBThreads / kMaxRun;  // item lanes per gradient slot
    const int t = threadIdx.x, T = blockDim.x;
    const BPass &P = A.passes[p];
    const BCirc &C = A.circs[P.circ];
    if (P.type == kPassAdj) {
        for (int v = t; v < kBThreads; v += T) {
            const int r = v % kMaxRun, lane = v / kMaxRun;
            double s = 0.0;
            if (r < P.count)
                for (int i = lane; i < P.nitems; i += LANES) s += A.gpart[C.gpart_off + (int64_t)i * kMaxRun + r];
            sh[v] = s;
        }
        __syncthreads();
        if (t < P.count) {
            double g = 0.0;
            for (int l = 0; l < LANES; ++l) g += sh[l * kMaxRun + t];
            A.grad[C.theta_off + A.rot[P.first + t].k] = g;
        }
        __syncthreads();
    }
    if (P.flags & kFlagEnergy) {
        for (int v = t; v < kBThreads; v += T) {
            double s = 0.0;
            if (v < kMaxRun)
                for (int i = v; i < P.nitems; i += kMaxRun) s += A.epart[C.epart_off + i];
            sh[v] = s;
        }
        __syncthreads();
        if (t == 0) {
            double e = 0.0;
            for (int l = 0; l < kMaxRun; ++l) e += sh[l];
            A.energy[P.circ] = e;
        }
        __syncthreads();
    }
    const bool ends = A.with_grad ? P.end_flag_grad : (P.flags & kFlagEnd);
    if (ends && t == 0) A.t_end[P.circ] = wall_clock64();
}

// Persistent runs (tuning variant 1): control words, cleared before each run.
// A dependency wait gives up after this long by default; a correct run's
// longest wait is about one pass of its largest circuit (milliseconds).
constexpr double kPersistWaitSeconds = 2.0;
enum { kCtlTicket = 0, kCtlAbort = 1, kCtlStatus = 2, kCtlWords = 4 };

struct PersistArgs {
    const BItem *tickets;   // work items in claim order
    const int32_t *prev;    // per pass: the pass before it in its circuit's chain, -1 for none
    uint32_t *done;         // per pass: items finished
    uint32_t *ready;        // per pass: 1 once its items are finished and its partial sums reduced
    uint32_t *ctl;          // kCtl* words
    uint64_t max_wait;      // a dependency wait gives up after this many wall-clock ticks
    int32_t nt;             // tickets
    uint32_t need;          // ready value a wait needs: 1 (2 is never written: every wait gives up)
};

// One launch runs every work item of a forward (grad = false: rotation and
// measurement passes) or gradient run (rotation, H psi and adjoint passes)
// on max_grid workgroups (0: as many as fit on the device at once); the grid
// used is returned in *grid_out.
template <typename Amp>
cfh_status launch_batch_persist(int reg_bits, bool grad, int max_grid, hipStream_t s, const BatchArgs &A,
                                const PassArgs2 *pa, const PersistArgs &Q, int *grid_out);
extern template cfh_status launch_batch_persist<double2>(int, bool, int, hipStream_t, const BatchArgs &,
                                                         const PassArgs2 *, const PersistArgs &, int *);
extern template cfh_status launch_batch_persist<float2>(int, bool, int, hipStream_t, const BatchArgs &,
                                                        const PassArgs2 *, const PersistArgs &, int *);

// Register-tiled forward rotation items of one level: one workgroup of
// 2^(b-4) threads per item, every item a range of cosets of one pass whose
// PassArgs2 is pa[passes[item.pass].p2].  The first pass of a circuit builds
// its basis state instead of reading psi.
constexpr int kBatchRegTile = 12;  // default register tile (tuning reg_tile_bits)
// A work item covers at most this many tiles.  A pass is cut into the tuned
// number of items (tuning batch_items), or into more when its tiles would
// exceed this bound, so that the passes of large circuits spread over the GPU
// even when such a circuit runs alone (a 30-qubit pass on 2^12 tiles: 4,096
// items instead of 32).  Circuits of up to 20 qubits never reach it.
constexpr uint64_t kBatchMaxTilesPerItem = 64;
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
