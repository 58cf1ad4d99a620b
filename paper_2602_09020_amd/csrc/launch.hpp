// Host-side launch helpers shared by the translation units of libcfh.
#pragma once

#include <hip/hip_runtime.h>

#include "cfh_internal.hpp"

namespace cfh {

// True on hipSuccess; otherwise records the HIP error as CFH_E_HIP in *st.
bool hip_ok(hipError_t e, const char *what, cfh_status *st);

// Status of the last kernel launch (clears the HIP error state).
cfh_status last_launch(const char *what);

// Persistent grid: as many workgroups as can be resident at once (cached per
// kernel, LDS size and device).
unsigned resident_grid(const void *fn, int threads, size_t lds);

// One register-tiled pass (k_pass2) over every coset of the pass's tile
// subspace.  mode bit 0 = prefetch the next coset, bit 1 = compile-time
// bodies, bit 2 = half-tile transposes, bit 3 = read-only measurement (adds
// each workgroup's share of sum_k w_k <P_k> to partial[workgroup]; at most
// max_grid workgroups when max_grid > 0).  Instantiated for double2 and float2
// storage in their own translation units.
template <typename Amp>
cfh_status launch_pass2(uint64_t ntiles, hipStream_t s, Amp *psi, const double2 *coef, const PassArgs2 &a,
                        int mode, double2 *partial = nullptr, unsigned max_grid = 0);
extern template cfh_status launch_pass2<double2>(uint64_t, hipStream_t, double2 *, const double2 *,
                                                 const PassArgs2 &, int, double2 *, unsigned);
extern template cfh_status launch_pass2<float2>(uint64_t, hipStream_t, float2 *, const double2 *,
                                                const PassArgs2 &, int, double2 *, unsigned);

// Register-tiled adjoint pass over every coset: rewinds psi and lam by the
// pass's rotations (inverse-order descriptors) and writes
// grad[k] = Im <lam|P_k|psi> for each of them (one reduction launch follows
// the pass).  gpart holds max_grid * kMaxRun doubles of scratch.
template <typename Amp>
cfh_status launch_adj2(uint64_t ntiles, hipStream_t s, Amp *psi, Amp *lam, const double2 *coef, const PassArgs2 &a,
                       bool half, double *gpart, unsigned max_grid, double *grad);
extern template cfh_status launch_adj2<double2>(uint64_t, hipStream_t, double2 *, double2 *, const double2 *,
                                                const PassArgs2 &, bool, double *, unsigned, double *);
extern template cfh_status launch_adj2<float2>(uint64_t, hipStream_t, float2 *, float2 *, const double2 *,
                                               const PassArgs2 &, bool, double *, unsigned, double *);

// Register-tiled H psi pass over every coset: lam (+)= sum_k w_k P_k psi over
// the pass's terms (w in device memory, indexed by the descriptors' k); lam
// is read only when accumulate is set.
template <typename Amp>
cfh_status launch_ham2(uint64_t ntiles, hipStream_t s, const Amp *psi, Amp *lam, const double2 *mw,
                       const PassArgs2 &a, int accumulate);
extern template cfh_status launch_ham2<double2>(uint64_t, hipStream_t, const double2 *, double2 *, const double2 *,
                                                const PassArgs2 &, int);
extern template cfh_status launch_ham2<float2>(uint64_t, hipStream_t, const float2 *, float2 *, const double2 *,
                                               const PassArgs2 &, int);

} // namespace cfh
